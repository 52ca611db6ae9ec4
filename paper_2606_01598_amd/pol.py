"""Python binding of the polarizable-model calls (include/pol.h), same names.

Tensors are torch HIP tensors (float32 contiguous per-atom arrays, a float64
(3, 3) device cell for the PME plan).  The model, its Thole damping and the
self-consistent solve run in the library's HIP kernels; this module checks
shapes and passes pointers and the current stream.

* ``PolPlan``              -- pol_plan_create / pol_plan_destroy
* ``PolPlan.real(...)``    -- pol_real: E_real, dE_real/dr, dE_real/dq, dE_real/dmu
* ``PolPlan.mixed(...)``   -- pol_real_mixed: d/dmu (grad_r E_real . v)
* ``PolPlan.model(...)``   -- pol_model: U(q, mu), dU/dr, dU/dq, dU/dmu
* ``PolPlan.model_hvp(...)`` -- pol_model_hvp: the q and mu rows of the model
  Hessian applied to (v_pos, v_q, v_mu)
* ``PolPlan.scf(...)``     -- pol_scf: induced dipoles by preconditioned CG
* ``teacher(...)``         -- pol_scf then pol_model: dipoles, energy and forces
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from .pme import _atoms, _ptr, _stream

THOLE_A = 0.39


class PolPlan:
    """Real-space Thole-damped Ewald terms and the induced-dipole solve for one cell."""

    def __init__(self, box, alpha: float, cutoff: float, max_atoms: int,
                 thole_a: float = THOLE_A, prefactor: float = 1.0, warm_start: bool = False,
                 fixed_iters: bool = False, device=None):
        self._lib = _lib.load()
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        b = np.asarray(box.detach().cpu() if isinstance(box, torch.Tensor) else box,
                       dtype=np.float64).reshape(9)
        d = _lib.PolDesc()
        d.max_atoms = int(max_atoms)
        d.flags = ((_lib.POL_F_WARM_START if warm_start else 0)
                   | (_lib.POL_F_FIXED_ITERS if fixed_iters else 0))
        for k in range(9):
            d.box[k] = float(b[k])
        d.alpha = float(alpha)
        d.cutoff = float(cutoff)
        d.thole_a = float(thole_a)
        d.prefactor = float(prefactor)
        self.max_atoms = int(max_atoms)
        h = ctypes.c_void_p()
        _lib.check(self._lib.pol_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._lib.pol_plan_destroy(h)
            self.handle = None

    def _common(self, pos, pol):
        n = int(pos.shape[0])
        if n > self.max_atoms:
            raise _lib.PMEError(_lib.PME_ECAPACITY, "more atoms than the plan's max_atoms")
        _atoms("pos", pos, n, 3, self.device)
        _atoms("pol", pol, n, 0, self.device)
        return n

    def real(self, pos, q, mu, pol, energy=True, dE_dpos=True, dE_dmu=True, dE_dq=False):
        n = self._common(pos, pol)
        if q is not None:
            _atoms("q", q, n, 0, self.device)
        if mu is not None:
            _atoms("mu", mu, n, 3, self.device)
        out = {}
        if energy:
            out["energy"] = torch.empty(1, dtype=torch.float64, device=self.device)
        if dE_dpos:
            out["dE_dpos"] = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        if dE_dmu:
            out["dE_dmu"] = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        if dE_dq:
            out["dE_dq"] = torch.empty(n, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.pol_real(self.handle, _stream(), n, _ptr(pos), _ptr(q), _ptr(mu),
                                      _ptr(pol), _ptr(out.get("energy")), _ptr(out.get("dE_dpos")),
                                      _ptr(out.get("dE_dq")), _ptr(out.get("dE_dmu"))))
        return out

    def mixed(self, pos, q, mu, pol, v_pos):
        n = self._common(pos, pol)
        _atoms("v_pos", v_pos, n, 3, self.device)
        g = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.pol_real_mixed(self.handle, _stream(), n, _ptr(pos), _ptr(q),
                                            _ptr(mu), _ptr(pol), _ptr(v_pos), _ptr(g)))
        return g

    def model(self, pme_plan, pos, q, mu, pol, box, energy=True, dU_dpos=True, dU_dmu=True,
              dU_dq=False):
        n = self._common(pos, pol)
        _atoms("q", q, n, 0, self.device)
        if mu is not None:
            _atoms("mu", mu, n, 3, self.device)
        out = {}
        if energy:
            out["energy"] = torch.empty(1, dtype=torch.float64, device=self.device)
        if dU_dpos:
            out["dU_dpos"] = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        if dU_dmu:
            out["dU_dmu"] = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        if dU_dq:
            out["dU_dq"] = torch.empty(n, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.pol_model(self.handle, pme_plan.handle, _stream(), n, _ptr(pos),
                                       _ptr(q), _ptr(mu), _ptr(pol), _ptr(box),
                                       _ptr(out.get("energy")), _ptr(out.get("dU_dpos")),
                                       _ptr(out.get("dU_dq")), _ptr(out.get("dU_dmu"))))
        return out

    def model_hvp(self, pme_plan, pos, q, mu, pol, box, v_pos=None, v_q=None, v_mu=None,
                  out=None):
        """pol_model_hvp: (g_q [n], g_mu [n, 3]), the q and mu rows of the Hessian of U
        applied to the tangent (v_pos, v_q, v_mu) (None = zero)."""
        n = self._common(pos, pol)
        _atoms("q", q, n, 0, self.device)
        for name, t, w in (("mu", mu, 3), ("v_pos", v_pos, 3), ("v_q", v_q, 0),
                           ("v_mu", v_mu, 3)):
            if t is not None:
                _atoms(name, t, n, w, self.device)
        o = out if out is not None else {
            "g_q": torch.empty(n, dtype=torch.float32, device=self.device),
            "g_mu": torch.empty(n, 3, dtype=torch.float32, device=self.device)}
        _lib.check(self._lib.pol_model_hvp(self.handle, pme_plan.handle, _stream(), n, _ptr(pos),
                                           _ptr(q), _ptr(mu), _ptr(pol), _ptr(box), _ptr(v_pos),
                                           _ptr(v_q), _ptr(v_mu), _ptr(o["g_q"]),
                                           _ptr(o["g_mu"])))
        return o

    def scf(self, pme_plan, pos, q, pol, box, tol: float = 1e-6, max_iter: int = 200,
            mu: Optional[torch.Tensor] = None):
        """Induced dipoles (n, 3), iterations and final RMS residual.  `mu`, when
        given, receives the solution (and is the initial guess of a warm-start plan)."""
        n = self._common(pos, pol)
        if mu is None:
            mu = torch.zeros(n, 3, dtype=torch.float32, device=self.device)
        it = ctypes.c_int32(0)
        res = ctypes.c_double(0.0)
        _lib.check(self._lib.pol_scf(self.handle, pme_plan.handle, _stream(), n, _ptr(pos),
                                     _ptr(q), _ptr(pol), _ptr(box), float(tol), int(max_iter),
                                     _ptr(mu), ctypes.byref(it), ctypes.byref(res)))
        return mu, int(it.value), float(res.value)


def teacher(pol_plan: PolPlan, pme_plan, pos, q, pol, box, tol: float = 1e-6,
            max_iter: int = 300):
    """Self-consistent dipoles and the model's energy and forces at them
    (dict: mu, energy, dU_dpos, iters, resid)."""
    mu, it, res = pol_plan.scf(pme_plan, pos, q, pol, box, tol=tol, max_iter=max_iter)
    out = pol_plan.model(pme_plan, pos, q, mu, pol, box, dU_dmu=False)
    out.update(mu=mu, iters=it, resid=res)
    return out
