"""Python binding of the batched calls (pme_batch_* of include/pme.h): many
boxes of uneven atom count and mesh evaluated by one launch per kernel kind,
and one training step of the whole batch captured as a HIP graph.

Per-atom tensors are packed (the atoms of box b follow those of box b-1),
cells are (nbox, 3, 3) float64 and energies (nbox, 3) float64.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .pme import _ptr, _stream


class Batch:
    def __init__(self, meshes, n_atoms, order: int, alpha: float, influence_power: float = 1.0,
                 prefactor: float = 1.0, tiles=None, device=None, fft_lines=None,
                 optimal_influence: bool = False):
        self._lib = _lib.load()
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        nbox = len(meshes)
        descs = (_lib.PMEDesc * nbox)()
        for b in range(nbox):
            d = descs[b]
            for k in range(3):
                d.mesh[k] = int(meshes[b][k])
                d.tile[k] = 0 if tiles is None else int(tiles[b][k])
            d.fft_lines = 0 if fft_lines is None else int(fft_lines[b])
            d.order = int(order)
            d.max_atoms = max(1, int(n_atoms[b]))
            d.flags = _lib.PME_F_KEEP_PHI | (_lib.PME_F_OPT_INFLUENCE if optimal_influence else 0)
            d.alpha = float(alpha)
            d.influence_power = float(influence_power)
            d.prefactor = float(prefactor)
        n = (ctypes.c_int32 * nbox)(*[int(v) for v in n_atoms])
        h = ctypes.c_void_p()
        _lib.check(self._lib.pme_batch_plan(descs, nbox, n, ctypes.byref(h)))
        self.handle = h
        self.nbox = nbox
        self.n_atoms = [int(v) for v in n_atoms]
        self.total = int(sum(self.n_atoms))
        self.offsets = np.concatenate([[0], np.cumsum(self.n_atoms)]).astype(int)
        self._step = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._lib.pme_batch_destroy(h)
            self.handle = None

    def _check(self, pos, box):
        if tuple(pos.shape) != (self.total, 3) or pos.dtype != torch.float32:
            raise ValueError("pos must be packed float32 (total, 3)")
        if tuple(box.shape) != (self.nbox, 3, 3) or box.dtype != torch.float64:
            raise ValueError("box must be float64 (nbox, 3, 3)")

    def _empty(self, *shape, dtype=torch.float32):
        return torch.empty(*shape, dtype=dtype, device=self.device)

    def forward(self, pos, q, mu, box, out=None):
        self._check(pos, box)
        o = out if out is not None else {
            "energy": self._empty(self.nbox, 3, dtype=torch.float64),
            "dE_dpos": self._empty(self.total, 3), "dE_dq": self._empty(self.total),
            "dE_dmu": self._empty(self.total, 3)}
        _lib.check(self._lib.pme_batch_forward(self.handle, _stream(), _ptr(pos), _ptr(q), _ptr(mu),
                                               _ptr(box), _ptr(o.get("energy")), _ptr(o.get("dE_dpos")),
                                               _ptr(o.get("dE_dq")), _ptr(o.get("dE_dmu"))))
        return o

    def backward(self, pos, q, mu, box, v_pos=None, v_q=None, v_mu=None, out=None):
        self._check(pos, box)
        o = out if out is not None else {
            "g_pos": self._empty(self.total, 3), "g_q": self._empty(self.total),
            "g_mu": self._empty(self.total, 3)}
        _lib.check(self._lib.pme_batch_backward(self.handle, _stream(), _ptr(pos), _ptr(q), _ptr(mu),
                                                _ptr(box), _ptr(v_pos), _ptr(v_q), _ptr(v_mu),
                                                _ptr(o.get("g_pos")), _ptr(o.get("g_q")),
                                                _ptr(o.get("g_mu"))))
        return o

    def capture(self, step: dict):
        """Capture forward + H v + force-loss H v of the batch into a HIP graph.
        `step` maps the pme_batch_step_t field names to tensors, which must stay
        alive (they are kept here) and at the same addresses while replaying."""
        st = _lib.BatchStep()
        for name, _ in _lib.BatchStep._fields_:
            t = step.get(name)
            setattr(st, name, None if t is None else t.data_ptr())
        torch.cuda.synchronize()
        _lib.check(self._lib.pme_batch_graph_capture(self.handle, ctypes.byref(st)))
        self._step = dict(step)

    def replay(self):
        _lib.check(self._lib.pme_batch_graph_launch(self.handle, _stream()))

    def status(self):
        _lib.check(self._lib.pme_batch_status(self.handle, _stream()))
