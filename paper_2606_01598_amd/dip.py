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
* ``DipPlan.features_jvp(...)``   -- dip_features_jvp (feature tangent along positions)
* ``DipPlan.charges(...)``        -- dip_charges (charge head, Eq. charge_pred)
* ``DipPlan.forward_jvp(...)``    -- dip_forward_jvp (dipoles and their tangent)
* ``DipPlan.backward_jvp(...)``   -- dip_backward_jvp (second-order parameter gradient)
* ``DipPlan.loss(...)``           -- dip_loss
* ``adam(...)``                   -- dip_adam
* ``Trainer``                     -- one training step per teacher box, with an
  optional charge head and on Hellmann-Feynman or conservative forces
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .pme import _atoms, _ptr, _stream

NPARAM = _lib.DIP_NPARAM
NQPARAM = _lib.DIP_NQPARAM


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

    def position_vjp(self, theta, pos, q, feat, vec, u, out=None, qtheta=None, c=None,
                     base=None):
        """dip_position_vjp: base + sum_i (d mu_i/d r_j)^T u_i + (d q_i/d r_j) c_i for
        every atom j (u or c may be None, not both; c needs the charge head qtheta)."""
        n = self._n(pos)
        for name, t, w in (("u", u, 3), ("c", c, 0), ("base", base, 3)):
            if t is not None:
                _atoms(name, t, n, w, self.device)
        g = out if out is not None else torch.empty(n, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_position_vjp(self.handle, _stream(), n, _ptr(theta),
                                              _ptr(qtheta), _ptr(pos), _ptr(q), _ptr(feat),
                                              _ptr(vec), _ptr(u), _ptr(c), _ptr(base), _ptr(g)))
        return g

    def features_jvp(self, pos, q, vec, v):
        """dip_features_jvp: (feat_dot [n, 34], vec_dot [n, 16, 3]) along positions v."""
        n = self._n(pos)
        _atoms("v", v, n, 3, self.device)
        fd = torch.empty(n, _lib.DIP_NFEAT, dtype=torch.float32, device=self.device)
        vd = torch.empty(n, _lib.DIP_NCH, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_features_jvp(self.handle, _stream(), n, _ptr(pos), _ptr(q),
                                              _ptr(vec), _ptr(v), _ptr(fd), _ptr(vd)))
        return fd, vd

    def charges(self, qtheta, z, feat, feat_dot=None, q=True, q_dot=False):
        """dip_charges: the charge head's q [n] (and q_dot [n] along feat_dot); returns
        q, q_dot or (q, q_dot) as requested."""
        n = int(feat.shape[0])
        _atoms("z", z, n, 0, self.device)
        qo = torch.empty(n, dtype=torch.float32, device=self.device) if q else None
        qd = torch.empty(n, dtype=torch.float32, device=self.device) if q_dot else None
        _lib.check(self._lib.dip_charges(self.handle, _stream(), n, _ptr(qtheta), _ptr(z),
                                         _ptr(feat), _ptr(feat_dot), _ptr(qo), _ptr(qd)))
        return (qo, qd) if q and q_dot else (qo if q else qd)

    def forward_jvp(self, theta, feat, vec, feat_dot, vec_dot, mu=True):
        """dip_forward_jvp: (mu, mu_dot), or mu_dot alone with mu=False."""
        n = int(feat.shape[0])
        m = torch.empty(n, 3, dtype=torch.float32, device=self.device) if mu else None
        md = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_forward_jvp(self.handle, _stream(), n, _ptr(theta), _ptr(feat),
                                             _ptr(vec), _ptr(feat_dot), _ptr(vec_dot), _ptr(m),
                                             _ptr(md)))
        return (m, md) if mu else md

    def backward_jvp(self, theta, qtheta, feat, vec, feat_dot, vec_dot, g_mu0=None, g_mu1=None,
                     u=None, g_q0=None, g_q1=None, c=None, out=None, qout=None):
        """dip_backward_jvp: parameter gradients (dipole head, charge head) from the
        cotangents on mu, mu_dot, q and q_dot; a head whose parameters are None is
        skipped."""
        n = int(feat.shape[0])
        g = None
        if theta is not None:
            g = out if out is not None else torch.empty(NPARAM, dtype=torch.float32,
                                                        device=self.device)
        gq = None
        if qtheta is not None:
            gq = qout if qout is not None else torch.empty(NQPARAM, dtype=torch.float32,
                                                           device=self.device)
        _lib.check(self._lib.dip_backward_jvp(self.handle, _stream(), n, _ptr(theta),
                                              _ptr(qtheta), _ptr(feat), _ptr(vec),
                                              _ptr(feat_dot), _ptr(vec_dot), _ptr(g_mu0),
                                              _ptr(g_mu1), _ptr(u), _ptr(g_q0), _ptr(g_q1),
                                              _ptr(c), _ptr(g), _ptr(gq)))
        return g, gq

    def loss(self, U_s, U_t, dUdr_s, dUdr_t, mu, mu_t, dUdmu_s, lE=1.0, lF=1.0, lmu=0.0,
             out=None, dUdq_s=None):
        n = int(mu.shape[0])
        o = out if out is not None else {
            "loss": torch.empty(1, dtype=torch.float64, device=self.device),
            "v_pos": torch.empty(n, 3, dtype=torch.float32, device=self.device),
            "g_mu": torch.empty(n, 3, dtype=torch.float32, device=self.device)}
        if dUdq_s is not None and "g_q" not in o:
            o["g_q"] = torch.empty(n, dtype=torch.float32, device=self.device)
        _lib.check(self._lib.dip_loss(self.handle, _stream(), n, _ptr(U_s), _ptr(U_t),
                                      _ptr(dUdr_s), _ptr(dUdr_t), _ptr(mu), _ptr(mu_t),
                                      _ptr(dUdmu_s), _ptr(dUdq_s), float(lE), float(lF),
                                      float(lmu), _ptr(o["loss"]), _ptr(o["v_pos"]),
                                      _ptr(o["g_mu"]),
                                      _ptr(o.get("g_q") if dUdq_s is not None else None)))
        return o


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    lib = _lib.load()
    _lib.check(lib.dip_adam(_stream(), int(theta.numel()), int(t), float(lr), float(beta1),
                            float(beta2), float(eps), _ptr(theta), _ptr(grad), _ptr(m), _ptr(v)))


class Trainer:
    """Training through the PME model: for a teacher box (pos, q, pol, feat, vec,
    U_t, dUdr_t, mu_t; q holds the formal charges) one step evaluates the
    student's charges and dipoles, its energy and forces, the loss, the cotangents
    of the heads' outputs (direct part + the Hessian rows of the model applied to
    the force cotangent and, for conservative forces, to the heads' tangents), the
    parameter gradient and an Adam update.

    * ``qtheta0``: initial charge-head parameters (None: charges fixed at q).
    * ``conservative``: train on F = -dU(r, q(r), mu(r))/dr (second order through
      the features and both networks) instead of the Hellmann-Feynman -dU/dr.

    The parameters live in one buffer, dipole head then charge head, so one Adam
    call updates both."""

    def __init__(self, dip: DipPlan, pol_plan, pme_plan, box, theta0, lr=2e-3, lE=1.0, lF=1.0,
                 lmu=0.0, warmup=0, decay=1.0, decay_steps=1000, qtheta0=None,
                 conservative=False):
        self.dip, self.pol, self.pme, self.box = dip, pol_plan, pme_plan, box
        dev = dip.device
        parts = [np.asarray(theta0, dtype=np.float64)]
        if qtheta0 is not None:
            parts.append(np.asarray(qtheta0, dtype=np.float64))
        self.params = torch.tensor(np.concatenate(parts), dtype=torch.float32, device=dev)
        self.theta = self.params[:NPARAM]
        self.qtheta = self.params[NPARAM:] if qtheta0 is not None else None
        self.charge_head = qtheta0 is not None
        self.conservative = bool(conservative)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.empty_like(self.params)
        self.g = self.grad[:NPARAM]
        self.gq = self.grad[NPARAM:] if self.charge_head else None
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

    def charges(self, b):
        """The student's charges for box b (the formal charges without a charge head)."""
        if not self.charge_head:
            return b["q"]
        return self.dip.charges(self.qtheta, b["q"], b["feat"])

    def evaluate(self, b):
        """Energy, forces -dU/dr (conservative when so trained), charges and dipoles."""
        q = self.charges(b)
        mu = self.dip.forward(self.theta, b["feat"], b["vec"])
        s = self.pol.model(self.pme, b["pos"], q, mu, b["pol"], self.box,
                           dU_dq=self.charge_head and self.conservative)
        G = s["dU_dpos"]
        if self.conservative:
            G = self.dip.position_vjp(self.theta, b["pos"], b["q"], b["feat"], b["vec"],
                                      s["dU_dmu"], qtheta=self.qtheta, c=s.get("dU_dq"),
                                      base=G)
        return {"energy": s["energy"], "dU_dpos": G, "q": q, "mu": mu}

    def step(self, b):
        if not (self.charge_head or self.conservative):
            return self._step_dipoles_hf(b)
        pos, z, feat, vec = b["pos"], b["q"], b["feat"], b["vec"]
        q = self.charges(b)
        mu = self.dip.forward(self.theta, feat, vec)
        s = self.pol.model(self.pme, pos, q, mu, b["pol"], self.box, dU_dq=self.charge_head)
        Uq = s.get("dU_dq")
        G = s["dU_dpos"]
        if self.conservative:
            G = self.dip.position_vjp(self.theta, pos, z, feat, vec, s["dU_dmu"],
                                      qtheta=self.qtheta, c=Uq, base=G)
        o = self.dip.loss(s["energy"], b["U"], G, b["dUdr"], mu, b.get("mu"), s["dU_dmu"],
                          self.lE, self.lF, self.lmu, dUdq_s=Uq)
        fd = vd = qd = mud = None
        if self.conservative:
            fd, vd = self.dip.features_jvp(pos, z, vec, o["v_pos"])
            if self.charge_head:
                qd = self.dip.charges(self.qtheta, z, feat, fd, q=False, q_dot=True)
            mud = self.dip.forward_jvp(self.theta, feat, vec, fd, vd, mu=False)
        h = self.pol.model_hvp(self.pme, pos, q, mu, b["pol"], self.box, o["v_pos"], qd, mud)
        cons = self.conservative
        self.dip.backward_jvp(self.theta, self.qtheta, feat, vec, fd, vd, o["g_mu"], h["g_mu"],
                              s["dU_dmu"] if cons else None, o.get("g_q"), h["g_q"],
                              Uq if cons else None, out=self.g, qout=self.gq)
        self.t += 1
        adam(self.params, self.grad, self.m, self.v, self.t, lr=self.rate(self.t))
        return o["loss"]

    def _step_dipoles_hf(self, b):
        mu = self.dip.forward(self.theta, b["feat"], b["vec"])
        s = self.pol.model(self.pme, b["pos"], b["q"], mu, b["pol"], self.box)
        o = self.dip.loss(s["energy"], b["U"], s["dU_dpos"], b["dUdr"], mu, b.get("mu"),
                          s["dU_dmu"], self.lE, self.lF, self.lmu)
        h_pme = self.pme.backward(b["pos"], b["q"], mu, self.box, o["v_pos"], None, None,
                                  g_pos=False, g_q=False)["g_mu"]
        h_real = self.pol.mixed(b["pos"], b["q"], mu, b["pol"], o["v_pos"])
        self.dip.backward(self.theta, b["feat"], b["vec"], o["g_mu"], h_pme, h_real, out=self.g)
        self.t += 1
        adam(self.params, self.grad, self.m, self.v, self.t, lr=self.rate(self.t))
        return o["loss"]
