"""Python binding of the learned dipole head (include/dip.h), same names, plus
the training loop through the PME model that strings the C calls together.

Every arithmetic step runs in the library's HIP kernels (features, network,
loss, the PME and real-space Hessian products, backpropagation, Adam); this
module allocates device buffers and passes pointers and the current stream.

* ``DipPlan``                     -- dip_plan_create / dip_plan_destroy
* ``DipPlan.features(pos, q)``    -- dip_features
* ``DipPlan.forward(theta, ...)`` -- dip_forward
* ``DipPlan.backward(...)``       -- dip_backward
* ``DipPlan.position_vjp(...)``   -- dip_position_vjp (conservative student forces)
* ``DipPlan.loss(...)``           -- dip_loss
* ``adam(...)``                   -- dip_adam
* ``Trainer``                     -- one training step per teacher box
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .pme import _atoms, _ptr, _stream

NPARAM = _lib.DIP_NPARAM


class DipPlan:
    def __init__(self, box, max_atoms: int, cutoff: float = 5.0, device=None):
        self._lib = _lib.load()
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        b = np.asarray(box.detach().cpu() if isinstance(box, torch.Tensor) else box,
                       dtype=np.float64).reshape(9)
        d = _lib.DipDesc()
        d.max_atoms = int(max_atoms)
        d.flags = 0
        for k in range(9):
            d.box[k] = float(b[k])
        d.cutoff = float(cutoff)
        self.max_atoms = int(max_atoms)
        h = ctypes.c_void_p()
        _lib.check(self._lib.dip_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._lib.dip_plan_destroy(h)
            self.handle = None

    def _n(self, pos):
        n = int(pos.shape[0])
        if n > self.max_atoms:
            raise _lib.PMEError(_lib.PME_ECAPACITY, "more atoms than the plan's max_atoms")
        _atoms("pos", pos, n, 3, self.device)
        return n

    def features(self, pos, q):
        n = self._n(pos)
        _atoms("q", q, n, 0, self.device)
        feat = torch.empty(n, _lib.DIP_NFEAT, dtype=torch.float32, device=self.device)
        vec = torch.empty(n, _lib.DIP_NCH, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_features(self.handle, _stream(), n, _ptr(pos), _ptr(q),
                                          _ptr(feat), _ptr(vec)))
        return feat, vec

    def forward(self, theta, feat, vec, out=None):
        n = int(feat.shape[0])
        mu = out if out is not None else torch.empty(n, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_forward(self.handle, _stream(), n, _ptr(theta), _ptr(feat),
                                         _ptr(vec), _ptr(mu)))
        return mu

    def backward(self, theta, feat, vec, g_mu0, g_mu1=None, g_mu2=None, out=None):
        n = int(feat.shape[0])
        g = out if out is not None else torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_backward(self.handle, _stream(), n, _ptr(theta), _ptr(feat),
                                          _ptr(vec), _ptr(g_mu0), _ptr(g_mu1), _ptr(g_mu2),
                                          _ptr(g)))
        return g

    def position_vjp(self, theta, pos, q, feat, vec, u, out=None):
        """dip_position_vjp: sum_i (d mu_i / d r_j)^T u_i for every atom j."""
        n = self._n(pos)
        _atoms("u", u, n, 3, self.device)
        g = out if out is not None else torch.empty(n, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_position_vjp(self.handle, _stream(), n, _ptr(theta), _ptr(pos),
                                              _ptr(q), _ptr(feat), _ptr(vec), _ptr(u), _ptr(g)))
        return g

    def loss(self, U_s, U_t, dUdr_s, dUdr_t, mu, mu_t, dUdmu_s, lE=1.0, lF=1.0, lmu=0.0,
             out=None):
        n = int(mu.shape[0])
        o = out if out is not None else {
            "loss": torch.empty(1, dtype=torch.float64, device=self.device),
            "v_pos": torch.empty(n, 3, dtype=torch.float32, device=self.device),
            "g_mu": torch.empty(n, 3, dtype=torch.float32, device=self.device)}
        _lib.check(self._lib.dip_loss(self.handle, _stream(), n, _ptr(U_s), _ptr(U_t),
                                      _ptr(dUdr_s), _ptr(dUdr_t), _ptr(mu), _ptr(mu_t),
                                      _ptr(dUdmu_s), float(lE), float(lF), float(lmu),
                                      _ptr(o["loss"]), _ptr(o["v_pos"]), _ptr(o["g_mu"])))
        return o


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    lib = _lib.load()
    _lib.check(lib.dip_adam(_stream(), int(theta.numel()), int(t), float(lr), float(beta1),
                            float(beta2), float(eps), _ptr(theta), _ptr(grad), _ptr(m), _ptr(v)))


class Trainer:
    """Training through the PME model: for a teacher box (pos, q, pol, feat, vec,
    U_t, dUdr_t, mu_t) one step evaluates the student's dipoles, its energy and
    forces, the loss, the dipole gradient (direct part + PME and real-space
    Hessian products with the force cotangent), the parameter gradient and an Adam
    update."""

    def __init__(self, dip: DipPlan, pol_plan, pme_plan, box, theta0, lr=2e-3, lE=1.0, lF=1.0,
                 lmu=0.0, warmup=0, decay=1.0, decay_steps=1000):
        self.dip, self.pol, self.pme, self.box = dip, pol_plan, pme_plan, box
        dev = dip.device
        self.theta = torch.tensor(np.asarray(theta0), dtype=torch.float32, device=dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.g = torch.empty_like(self.theta)
        self.t = 0
        self.lr, self.lE, self.lF, self.lmu = lr, lE, lF, lmu
        self.warmup, self.decay, self.decay_steps = int(warmup), float(decay), float(decay_steps)

    def rate(self, t: int) -> float:
        """Learning rate of step t (1-based): a linear warmup over `warmup` steps, then
        exponential decay by `decay` every `decay_steps` steps (the optimizer setting
        of Sec. 2.4: Adam with warmup and exponential decay)."""
        warm = min(1.0, t / self.warmup) if self.warmup > 0 else 1.0
        return self.lr * warm * self.decay ** (max(0, t - self.warmup) / self.decay_steps)

    def predict(self, feat, vec):
        return self.dip.forward(self.theta, feat, vec)

    def step(self, b):
        mu = self.dip.forward(self.theta, b["feat"], b["vec"])
        s = self.pol.model(self.pme, b["pos"], b["q"], mu, b["pol"], self.box)
        o = self.dip.loss(s["energy"], b["U"], s["dU_dpos"], b["dUdr"], mu, b.get("mu"),
                          s["dU_dmu"], self.lE, self.lF, self.lmu)
        h_pme = self.pme.backward(b["pos"], b["q"], mu, self.box, o["v_pos"], None, None,
                                  g_pos=False, g_q=False)["g_mu"]
        h_real = self.pol.mixed(b["pos"], b["q"], mu, b["pol"], o["v_pos"])
        self.dip.backward(self.theta, b["feat"], b["vec"], o["g_mu"], h_pme, h_real, out=self.g)
        self.t += 1
        adam(self.theta, self.g, self.m, self.v, self.t, lr=self.rate(self.t))
        return o["loss"]
