"""Python binding of the PME library with the same names as the C ABI.

Tensors are torch CUDA (HIP) tensors: float32 contiguous for atoms, float64
(3, 3) for the cell.  Every step of the computation runs in the library's HIP
kernels; this module only checks shapes and passes pointers and the current
stream.

* ``mesh_dims(box, spacing, strategy)``        -- Eq. mesh_target + strategies
* ``Plan``                                     -- pme_plan / destroy
* ``Plan.forward(...)``                        -- pme_forward (``cell=True``: pme_forward_cell,
  also dE/dbox at fixed Cartesian inputs)
* ``Plan.backward(...)``                       -- pme_backward (Hessian-vector product)
* ``Plan.step(...)``                           -- pme_step (forward and H v in one call)
* ``pme_energy(pos, q, mu, box, plan)``        -- E^lr as a differentiable torch op
  (first and second order: forces inside a loss, trained with create_graph)
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib

EV_PER_E2_ANGSTROM = 14.3996454784


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def mesh_dims(box, spacing: float, strategy: str = "smooth"):
    """Mesh dimensions of Eq. mesh_target mapped by 'pow2' | 'smooth' | 'ceil'."""
    lib = _lib.load()
    codes = {"pow2": _lib.PME_MESH_POW2, "smooth": _lib.PME_MESH_SMOOTH, "ceil": _lib.PME_MESH_CEIL}
    if strategy not in codes:
        raise ValueError(strategy)
    b = (ctypes.c_double * 9)(*[float(x) for x in torch.as_tensor(box, dtype=torch.float64).reshape(-1).tolist()])
    out = (ctypes.c_int32 * 3)()
    _lib.check(lib.pme_mesh_dims(b, float(spacing), codes[strategy], out))
    return tuple(int(x) for x in out)


def _atoms(name, t, n, cols, device):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.device.type == "cuda"):
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    shape = (n, cols) if cols else (n,)
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


class Plan:
    """A PME plan: mesh, order, alpha and the device workspaces (pme_plan)."""

    def __init__(self, mesh, order: int, alpha: float, max_atoms: int, influence_power: float = 1.0,
                 prefactor: float = 1.0, keep_phi: bool = True, device=None, tile=None,
                 concurrent: bool = False, optimal_influence: bool = False, fft_lines=None,
                 separate_spread: bool = False):
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        d = _lib.PMEDesc()
        for k in range(3):
            d.mesh[k] = int(mesh[k])
        d.order = int(order)
        d.max_atoms = int(max_atoms)
        d.flags = ((_lib.PME_F_KEEP_PHI if keep_phi else 0) | (_lib.PME_F_CONCURRENT if concurrent else 0)
                   | (_lib.PME_F_OPT_INFLUENCE if optimal_influence else 0)
                   | (_lib.PME_F_SEPARATE_SPREAD if separate_spread else 0))
        d.alpha = float(alpha)
        d.influence_power = float(influence_power)
        d.prefactor = float(prefactor)
        for k in range(3):
            d.tile[k] = 0 if tile is None else int(tile[k])
        d.fft_lines = 0 if fft_lines is None else int(fft_lines)
        self.desc = d
        self.mesh = tuple(int(m) for m in mesh)
        self.order = int(order)
        self.alpha = float(alpha)
        self.max_atoms = int(max_atoms)
        self.prefactor = float(prefactor)
        self.influence_power = float(influence_power)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.pme_plan(ctypes.byref(d), ctypes.byref(handle)))
        self.handle = handle

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._lib.pme_plan_destroy(h)
            self.handle = None

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.pme_plan_workspace_bytes(self.handle))

    def _check_common(self, pos, q, mu, box):
        if not (isinstance(pos, torch.Tensor) and pos.dim() == 2 and pos.shape[1] == 3):
            raise ValueError("pos must be (N, 3)")
        n = int(pos.shape[0])
        _atoms("pos", pos, n, 3, self.device)
        _atoms("q", q, n, 0, self.device)
        _atoms("mu", mu, n, 3, self.device)
        if not (isinstance(box, torch.Tensor) and box.device == self.device
                and box.dtype == torch.float64 and box.is_contiguous() and box.numel() == 9):
            raise TypeError("box must be a contiguous float64 (3, 3) tensor on the plan's device")
        return n

    def forward(self, pos, q, mu, box, energy=True, dE_dpos=True, dE_dq=True, dE_dmu=True,
                out=None, cell=False, theta=None):
        """pme_forward.  Returns dict(energy (3,) f64, dE_dpos, dE_dq, dE_dmu) of the
        requested outputs; ``out`` may supply preallocated tensors with those keys.
        With ``cell=True`` (pme_forward_cell) also dE_dbox (3, 3) f64, the gradient of
        E^lr with respect to the cell at fixed Cartesian positions.  With ``theta``
        (n, 6) float32 second moments (xx yy zz xy xz yz; pme_forward_quad) the energy
        has a fourth entry, the Theta self term, and dE_dtheta (n, 6) is added."""
        n = self._check_common(pos, q, mu, box)
        out = {} if out is None else dict(out)
        dev = self.device
        if theta is not None:
            if cell:
                raise ValueError("no cell gradient with quadrupoles")
            _atoms("theta", theta, n, 6, dev)
            if energy and "energy" not in out:
                out["energy"] = torch.empty(4, dtype=torch.float64, device=dev)
            if "dE_dtheta" not in out:
                out["dE_dtheta"] = torch.empty(n, 6, dtype=torch.float32, device=dev)
        if cell and "dE_dbox" not in out:
            out["dE_dbox"] = torch.empty(3, 3, dtype=torch.float64, device=dev)
        if energy and "energy" not in out:
            out["energy"] = torch.empty(3, dtype=torch.float64, device=dev)
        if dE_dpos and "dE_dpos" not in out:
            out["dE_dpos"] = torch.empty(n, 3, dtype=torch.float32, device=dev)
        if dE_dq and "dE_dq" not in out:
            out["dE_dq"] = torch.empty(n, dtype=torch.float32, device=dev)
        if dE_dmu and "dE_dmu" not in out:
            out["dE_dmu"] = torch.empty(n, 3, dtype=torch.float32, device=dev)
        args = (self.handle, _stream(), n, _ptr(pos), _ptr(q), _ptr(mu), _ptr(box),
                _ptr(out.get("energy")), _ptr(out.get("dE_dpos")), _ptr(out.get("dE_dq")),
                _ptr(out.get("dE_dmu")))
        if theta is not None:
            rc = self._lib.pme_forward_quad(self.handle, _stream(), n, _ptr(pos), _ptr(q), _ptr(mu),
                                            _ptr(theta), _ptr(box), _ptr(out.get("energy")),
                                            _ptr(out.get("dE_dpos")), _ptr(out.get("dE_dq")),
                                            _ptr(out.get("dE_dmu")), _ptr(out.get("dE_dtheta")))
        elif cell:
            rc = self._lib.pme_forward_cell(*args, _ptr(out["dE_dbox"]))
        else:
            rc = self._lib.pme_forward(*args)
        _lib.check(rc)
        return out

    def backward(self, pos, q, mu, box, v_pos=None, v_q=None, v_mu=None, g_pos=True, g_q=True,
                 g_mu=True, out=None):
        """pme_backward: Hessian-vector product H (v_pos, v_q, v_mu).  Returns dict."""
        n = self._check_common(pos, q, mu, box)
        _atoms("v_pos", v_pos, n, 3, self.device)
        _atoms("v_q", v_q, n, 0, self.device)
        _atoms("v_mu", v_mu, n, 3, self.device)
        out = {} if out is None else dict(out)
        dev = self.device
        if g_pos and "g_pos" not in out:
            out["g_pos"] = torch.empty(n, 3, dtype=torch.float32, device=dev)
        if g_q and "g_q" not in out:
            out["g_q"] = torch.empty(n, dtype=torch.float32, device=dev)
        if g_mu and "g_mu" not in out:
            out["g_mu"] = torch.empty(n, 3, dtype=torch.float32, device=dev)
        rc = self._lib.pme_backward(self.handle, _stream(), n, _ptr(pos), _ptr(q), _ptr(mu), _ptr(box),
                                    _ptr(v_pos), _ptr(v_q), _ptr(v_mu), _ptr(out.get("g_pos")),
                                    _ptr(out.get("g_q")), _ptr(out.get("g_mu")))
        _lib.check(rc)
        return out

    def step(self, pos, q, mu, box, v_pos=None, v_q=None, v_mu=None, out=None):
        """pme_step: forward outputs (energy, dE_dpos, dE_dq, dE_dmu) and the
        Hessian-vector product (g_pos, g_q, g_mu) of one evaluation, in one dict."""
        n = self._check_common(pos, q, mu, box)
        _atoms("v_pos", v_pos, n, 3, self.device)
        _atoms("v_q", v_q, n, 0, self.device)
        _atoms("v_mu", v_mu, n, 3, self.device)
        out = {} if out is None else dict(out)
        dev = self.device
        shapes = {"energy": ((3,), torch.float64), "dE_dpos": ((n, 3), torch.float32),
                  "dE_dq": ((n,), torch.float32), "dE_dmu": ((n, 3), torch.float32),
                  "g_pos": ((n, 3), torch.float32), "g_q": ((n,), torch.float32),
                  "g_mu": ((n, 3), torch.float32)}
        for k, (shape, dt) in shapes.items():
            if k not in out:
                out[k] = torch.empty(shape, dtype=dt, device=dev)
        rc = self._lib.pme_step(self.handle, _stream(), n, _ptr(pos), _ptr(q), _ptr(mu), _ptr(box),
                                _ptr(out["energy"]), _ptr(out["dE_dpos"]), _ptr(out["dE_dq"]),
                                _ptr(out["dE_dmu"]), _ptr(v_pos), _ptr(v_q), _ptr(v_mu),
                                _ptr(out["g_pos"]), _ptr(out["g_q"]), _ptr(out["g_mu"]))
        _lib.check(rc)
        return out

    def step_capture(self, steps, pos, q, mu, box, v_pos=None, v_q=None, v_mu=None, out=None):
        """pme_step_capture: capture ``steps`` pme_step calls into the plan's HIP graph
        (nothing runs).  Returns the output dict the replays write; the plan keeps the
        input and output tensors alive while the graph exists."""
        n = self._check_common(pos, q, mu, box)
        _atoms("v_pos", v_pos, n, 3, self.device)
        _atoms("v_q", v_q, n, 0, self.device)
        _atoms("v_mu", v_mu, n, 3, self.device)
        out = {} if out is None else dict(out)
        shapes = {"energy": ((3,), torch.float64), "dE_dpos": ((n, 3), torch.float32),
                  "dE_dq": ((n,), torch.float32), "dE_dmu": ((n, 3), torch.float32),
                  "g_pos": ((n, 3), torch.float32), "g_q": ((n,), torch.float32),
                  "g_mu": ((n, 3), torch.float32)}
        for k, (shape, dt) in shapes.items():
            if k not in out:
                out[k] = torch.empty(shape, dtype=dt, device=self.device)
        rc = self._lib.pme_step_capture(self.handle, int(steps), n, _ptr(pos), _ptr(q), _ptr(mu),
                                        _ptr(box), _ptr(out["energy"]), _ptr(out["dE_dpos"]),
                                        _ptr(out["dE_dq"]), _ptr(out["dE_dmu"]), _ptr(v_pos),
                                        _ptr(v_q), _ptr(v_mu), _ptr(out["g_pos"]), _ptr(out["g_q"]),
                                        _ptr(out["g_mu"]))
        _lib.check(rc)
        self._graph_refs = (pos, q, mu, box, v_pos, v_q, v_mu, out)
        return out

    def step_replay(self) -> None:
        """pme_step_replay on the current stream."""
        _lib.check(self._lib.pme_step_replay(self.handle, _stream()))

    def phi_id(self) -> int:
        """pme_plan_phi_id: identifier of the evaluation whose phi the plan keeps."""
        return int(self._lib.pme_plan_phi_id(self.handle))

    def drop_phi(self) -> None:
        """pme_plan_drop_phi: the next backward recomputes phi from its own inputs."""
        _lib.check(self._lib.pme_plan_drop_phi(self.handle))

    def status(self) -> None:
        """pme_status: synchronise and raise on device-detected errors."""
        _lib.check(self._lib.pme_status(self.handle, _stream()))

    def timer(self, kind) -> None:
        """pme_plan_timer: bracket every later launch of one kernel kind (a name of
        _lib.KERNEL_KINDS, or None to stop) with HIP events on the launch stream."""
        k = -1 if kind is None else _lib.KERNEL_KINDS.index(kind)
        _lib.check(self._lib.pme_plan_timer(self.handle, k))

    def timer_read(self):
        """pme_plan_timer_read: (launches, total milliseconds) since the last read."""
        import ctypes as ct
        n = ct.c_int64(0)
        ms = ct.c_double(0.0)
        _lib.check(self._lib.pme_plan_timer_read(self.handle, ct.byref(n), ct.byref(ms)))
        return int(n.value), float(ms.value)

    def phi(self) -> torch.Tensor:
        """Copy of the potential mesh of the last forward (N_x, N_y, N_z)."""
        return self._mesh_copy(self._lib.pme_plan_phi(self.handle))

    @property
    def spread_kind(self) -> str:
        """How the plan spreads the density: "tile", "band" or "fused"."""
        k = self._lib.pme_plan_spread_kind(self.handle)
        return {_lib.PME_SPREAD_TILE: "tile", _lib.PME_SPREAD_BAND: "band",
                _lib.PME_SPREAD_FUSED: "fused"}[k]

    def rho(self) -> torch.Tensor:
        """Copy of the last density spread (forward density or tangent density).
        A plan with the fused plane spread keeps no density mesh."""
        ptr = self._lib.pme_plan_rho(self.handle)
        if not ptr:
            raise RuntimeError("this plan spreads by x-planes fused with the transform and keeps "
                               "no density mesh; create it with separate_spread=True")
        return self._mesh_copy(ptr)

    def _mesh_copy(self, ptr) -> torch.Tensor:
        out = torch.empty(self.mesh, dtype=torch.float32, device=self.device)
        torch.cuda.current_stream().synchronize()
        nbytes = out.numel() * 4
        import ctypes as ct
        hip = ct.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_int]
        rc = hip.hipMemcpy(ct.c_void_p(out.data_ptr()), ct.c_void_p(ptr), nbytes, 3)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")
        return out


# -----------------------------------------------------------------------------
# autograd: E^lr(pos, q, mu) with hand-written first and second derivatives
# -----------------------------------------------------------------------------

class _PMEGrad(torch.autograd.Function):
    """(dE/dpos, dE/dq, dE/dmu) as a differentiable function of (pos, q, mu).

    Its backward is the Hessian-vector product of pme_backward, which is what a
    force loss needs when the forces were taken with create_graph=True.  The plan
    keeps the potential of its last evaluation; ``phi_id`` names the evaluation
    of these inputs, and when the plan has evaluated other inputs since (several
    frames of a batch loss through one plan), the kept potential is dropped so
    that pme_backward recomputes it from these inputs.
    """

    @staticmethod
    def forward(ctx, pos, q, mu, box, plan, phi_id, g_pos, g_q, g_mu):
        ctx.plan = plan
        ctx.phi_id = phi_id
        ctx.save_for_backward(pos, q, mu, box)
        return g_pos, g_q, g_mu

    @staticmethod
    def backward(ctx, v_pos, v_q, v_mu):
        pos, q, mu, box = ctx.saved_tensors
        plan = ctx.plan
        if plan.phi_id() != ctx.phi_id:
            plan.drop_phi()
        v = [None if t is None else t.contiguous().float() for t in (v_pos, v_q, v_mu)]
        r = plan.backward(pos.detach(), q.detach(), mu.detach(), box, *v)
        return r["g_pos"], r["g_q"], r["g_mu"], None, None, None, None, None, None


class _PMEEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, mu, box, plan):
        cell = box.requires_grad
        r = plan.forward(pos.detach(), q.detach(), mu.detach(), box.detach(), cell=cell)
        ctx.plan = plan
        ctx.phi_id = plan.phi_id()
        gb = r["dE_dbox"] if cell else torch.zeros(0, dtype=torch.float64, device=box.device)
        ctx.save_for_backward(pos, q, mu, box, r["dE_dpos"], r["dE_dq"], r["dE_dmu"], gb)
        return r["energy"].sum()

    @staticmethod
    def backward(ctx, gE):
        pos, q, mu, box, gp, gq, gm, gb = ctx.saved_tensors
        if torch.is_grad_enabled():
            gp, gq, gm = _PMEGrad.apply(pos, q, mu, box.detach(), ctx.plan, ctx.phi_id, gp, gq, gm)
        s = gE.to(torch.float32)
        # the cell gradient is first order: a constant for a second differentiation
        g_box = gb * gE.to(torch.float64) if gb.numel() else None
        return gp * s, gq * s, gm * s, g_box, None


class _PMEEnergyQuad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, mu, theta, box, plan):
        r = plan.forward(pos.detach(), q.detach(), mu.detach(), box.detach(),
                         theta=theta.detach())
        ctx.save_for_backward(r["dE_dpos"], r["dE_dq"], r["dE_dmu"], r["dE_dtheta"])
        return r["energy"].sum()

    @staticmethod
    def backward(ctx, gE):
        gp, gq, gm, gt = ctx.saved_tensors
        s = gE.to(torch.float32)
        return gp * s, gq * s, gm * s, gt * s, None, None


def pme_energy(pos: torch.Tensor, q: torch.Tensor, mu: torch.Tensor, box: torch.Tensor,
               plan: Plan, theta: torch.Tensor = None) -> torch.Tensor:
    """E^lr (float64 scalar) with gradients to pos, q and mu, differentiable twice, and
    to box (first order, pme_forward_cell) when box requires grad.  With second moments
    ``theta`` (n, 6; pme_forward_quad) the gradients to pos, q, mu and theta are first
    order (no Hessian-vector product for the quadrupole channel) and box takes none."""
    if theta is not None:
        if box.requires_grad:
            raise ValueError("no cell gradient with quadrupoles")
        return _PMEEnergyQuad.apply(pos, q, mu, theta, box, plan)
    return _PMEEnergy.apply(pos, q, mu, box, plan)
