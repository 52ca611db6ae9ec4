"""GPU parity of the charge head and of training on conservative forces
(include/dip.h: dip_charges, dip_features_jvp, dip_forward_jvp, dip_position_vjp
with both heads, dip_backward_jvp; include/pol.h: the dE/dq outputs and
pol_model_hvp) against the FP64 oracle (oracle/heads.py, oracle/pol.py), through
the C ABI.

Bar: relative RMS error <= 1e-4 (RMS_REL_TOL) of every per-atom output and
parameter gradient; relative error <= 1e-4 of the loss.  Network-only calls take
seeded synthetic feature arrays, so their sizes can pass the tile and workgroup
caps (8 and 16 atoms per tile, 512 workgroups) with ragged tails.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import RMS_REL_TOL, dev, f32, host, rel, rms_rel
from oracle import dip as odip
from oracle import heads as oh
from oracle import pol as opol

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev())


def _features(n, seed):
    """Seeded stand-ins for network inputs: positive scalar features, the species
    one-hot, vector channels and their tangents."""
    rng = np.random.default_rng(seed)
    x = np.abs(rng.normal(0.0, 0.7, (n, odip.NFEAT)))
    cat = rng.random(n) < 0.5
    x[:, 2 * odip.NCH] = cat
    x[:, 2 * odip.NCH + 1] = ~cat
    V = rng.normal(0.0, 0.5, (n, odip.NCH, 3))
    xd = rng.normal(0.0, 0.3, (n, odip.NFEAT))
    xd[:, 2 * odip.NCH:] = 0.0
    Vd = rng.normal(0.0, 0.3, (n, odip.NCH, 3))
    z = np.where(cat, 1.0, -1.0)
    return f32(x), f32(V), f32(xd), f32(Vd), z


def _plan(n, L=30.0):
    from paper_2606_01598_amd.dip import DipPlan
    return DipPlan(np.eye(3) * L, n, cutoff=5.0)


def _params(seed):
    return (f32(synth.mlp_init(seed, last_scale=1.0)),
            f32(synth.charge_head_init(seed + 1, last_scale=1.0, bias_scale=0.5)))


def test_pol_charge_gradients_parity():
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f = synth.molten_box(300, 41)
    pol = np.where(f.q > 0, 0.15, 3.5)
    mesh, p, alpha, rc = (24, 24, 24), 6, 0.35, 6.0
    rng = np.random.default_rng(1)
    q = f32(f.q + 0.2 * rng.normal(size=f.n))
    mu = f32(f.mu)
    pos, a = f32(f.pos), f32(pol)
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    out = plan.real(_t(pos), _t(q), _t(mu), _t(a), energy=False, dE_dpos=False, dE_dmu=False,
                    dE_dq=True)
    e_r = rms_rel(host(out["dE_dq"]), opol.real_charge_grad(pos, q, mu, f.box, alpha, rc, a))
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pme = Plan(mesh, p, alpha, max_atoms=f.n)
    m = plan.model(pme, _t(pos), _t(q), _t(mu), _t(a), box, dU_dq=True)
    U, Ur, Uq, Umu = opol.model_grads(pos, q, mu, f.box, mesh, p, alpha, rc, a)
    e_q, e_m = rms_rel(host(m["dU_dq"]), Uq), rms_rel(host(m["dU_dmu"]), Umu)
    e_u = rel(float(host(m["energy"])[0]), U)
    print("pol dq", f"real {e_r:.2e} model {e_q:.2e} mu {e_m:.2e} U {e_u:.2e}", flush=True)
    assert max(e_r, e_q, e_m) <= RMS_REL_TOL and e_u <= 1e-5


@pytest.mark.parametrize("which", ["r", "q", "mu", "all"])
def test_pol_model_hvp_parity(which):
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f = synth.molten_box(256, 42)
    pol = np.where(f.q > 0, 0.15, 3.5)
    mesh, p, alpha, rc = (24, 24, 24), 6, 0.35, 6.0
    rng = np.random.default_rng(2)
    n = f.n
    q = f32(f.q + 0.2 * rng.normal(size=n))
    pos, mu, a = f32(f.pos), f32(f.mu), f32(pol)
    vp = f32(rng.normal(size=(n, 3))) if which in ("r", "all") else None
    vq = f32(rng.normal(size=n)) if which in ("q", "all") else None
    vm = f32(rng.normal(size=(n, 3))) if which in ("mu", "all") else None
    print(f"case: pol_model_hvp n={n} tangents={which}", flush=True)
    plan = PolPlan(f.box, alpha, rc, max_atoms=n)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pme = Plan(mesh, p, alpha, max_atoms=n)
    h = plan.model_hvp(pme, _t(pos), _t(q), _t(mu), _t(a), box,
                       None if vp is None else _t(vp), None if vq is None else _t(vq),
                       None if vm is None else _t(vm))
    r_q, r_mu = opol.model_hvp(pos, q, mu, f.box, mesh, p, alpha, rc, a, vp, vq, vm)
    e_q, e_m = rms_rel(host(h["g_q"]), r_q), rms_rel(host(h["g_mu"]), r_mu)
    print("hvp", which, f"q {e_q:.2e} mu {e_m:.2e}", flush=True)
    assert e_q <= RMS_REL_TOL and e_m <= RMS_REL_TOL


def test_features_jvp_parity():
    from paper_2606_01598_amd.dip import DipPlan
    f = synth.molten_box(300, 43)
    plan = DipPlan(f.box, f.n, cutoff=5.0)
    pos, q = f32(f.pos), f32(f.q)
    v = f32(np.random.default_rng(3).normal(size=(f.n, 3)))
    feat, vec = plan.features(_t(pos), _t(q))
    fd, vd = plan.features_jvp(_t(pos), _t(q), vec, _t(v))
    xd, Vd = oh.features_jvp(pos, q, f.box, 5.0, v)
    e1, e2 = rms_rel(host(fd), xd), rms_rel(host(vd), Vd)
    print("features_jvp", f"{e1:.2e}", f"{e2:.2e}", flush=True)
    assert e1 <= RMS_REL_TOL and e2 <= RMS_REL_TOL
    assert torch.all(fd[:, 2 * odip.NCH:] == 0)


@pytest.mark.parametrize("n", [1, 37, 4099])
def test_charges_parity(n):
    x, _, xd, _, z = _features(n, 50 + n)
    _, thq = _params(7)
    plan = _plan(n)
    q, qd = plan.charges(_t(thq), _t(z), _t(x), _t(xd), q=True, q_dot=True)
    q_ref, qd_ref = oh.charges(thq, x, z, xd)
    e_q = rms_rel(host(q) - z, q_ref - z, floor=1e-3)
    e_d = rms_rel(host(qd), qd_ref, floor=1e-3)
    print("charges", n, f"{e_q:.2e}", f"{e_d:.2e}", flush=True)
    assert e_q <= RMS_REL_TOL and e_d <= RMS_REL_TOL
    # neutrality: the corrections sum to zero up to FP32 rounding
    assert abs(float(host(q).sum() - z.sum())) <= 1e-5 * n
    # without feat_dot the tangent is zero and q is unchanged
    q2 = plan.charges(_t(thq), _t(z), _t(x))
    assert torch.equal(q2, q)


@pytest.mark.parametrize("n", [5, 37, 4099])
def test_forward_jvp_parity(n):
    x, V, xd, Vd, _ = _features(n, 60 + n)
    theta, _ = _params(8)
    plan = _plan(n)
    mu, mud = plan.forward_jvp(_t(theta), _t(x), _t(V), _t(xd), _t(Vd))
    mu_ref, mud_ref, _, _, _ = oh.dipoles_jvp(theta, x, V, xd, Vd)
    e1, e2 = rms_rel(host(mu), mu_ref), rms_rel(host(mud), mud_ref)
    print("forward_jvp", n, f"{e1:.2e}", f"{e2:.2e}", flush=True)
    assert e1 <= RMS_REL_TOL and e2 <= RMS_REL_TOL
    # the primal part is dip_forward's
    assert rms_rel(host(plan.forward(_t(theta), _t(x), _t(V))), host(mu)) <= 1e-6


@pytest.mark.parametrize("n", [3, 37, 5001])
def test_backward_jvp_parity(n):
    x, V, xd, Vd, _ = _features(n, 70 + n)
    theta, thq = _params(9)
    rng = np.random.default_rng(n)
    g0, g1, u = (f32(rng.normal(size=(n, 3))) for _ in range(3))
    gq0, gq1, c = (f32(rng.normal(size=n)) for _ in range(3))
    plan = _plan(n)
    print(f"case: dip_backward_jvp n={n}", flush=True)
    g, gq = plan.backward_jvp(_t(theta), _t(thq), _t(x), _t(V), _t(xd), _t(Vd), _t(g0), _t(g1),
                              _t(u), _t(gq0), _t(gq1), _t(c))
    gw = np.einsum('nd,ncd->nc', g0 + g1, V) + np.einsum('nd,ncd->nc', u, Vd)
    gwd = np.einsum('nd,ncd->nc', u, V)
    g_ref = oh.mlp_jvp_backward(theta, oh.mlp_jvp(theta, x, xd)[2], gw, gwd)
    gq_ref = oh.charge_jvp_backward(thq, oh.charge_jvp(thq, x, xd)[2], oh.centre(gq0 + gq1),
                                    oh.centre(c))
    e1, e2 = rms_rel(host(g), g_ref), rms_rel(host(gq), gq_ref)
    print("backward_jvp", n, f"{e1:.2e}", f"{e2:.2e}", flush=True)
    assert e1 <= RMS_REL_TOL and e2 <= RMS_REL_TOL
    # no tangents: the first-order gradient of dip_backward
    g_fo, _ = plan.backward_jvp(_t(theta), None, _t(x), _t(V), None, None, _t(g0), _t(g1), _t(u))
    g_b = plan.backward(_t(theta), _t(x), _t(V), _t(g0), _t(g1))
    assert rms_rel(host(g_fo), host(g_b)) <= 1e-6
    # deterministic
    g2, gq2 = plan.backward_jvp(_t(theta), _t(thq), _t(x), _t(V), _t(xd), _t(Vd), _t(g0),
                                _t(g1), _t(u), _t(gq0), _t(gq1), _t(c))
    assert torch.equal(g, g2) and torch.equal(gq, gq2)


def test_position_vjp_both_heads_parity():
    from paper_2606_01598_amd.dip import DipPlan
    f = synth.molten_box(300, 44)
    plan = DipPlan(f.box, f.n, cutoff=5.0)
    pos, z = f32(f.pos), f32(f.q)
    theta, thq = _params(10)
    rng = np.random.default_rng(5)
    u, c, base = f32(rng.normal(size=(f.n, 3))), f32(rng.normal(size=f.n)), f32(rng.normal(size=(f.n, 3)))
    feat, vec = plan.features(_t(pos), _t(z))
    g = plan.position_vjp(_t(theta), _t(pos), _t(z), feat, vec, _t(u), qtheta=_t(thq), c=_t(c),
                          base=_t(base))
    g_ref = base + oh.position_vjp(theta, thq, pos, z, f.box, 5.0, u, c)
    gc = plan.position_vjp(None, _t(pos), _t(z), feat, vec, None, qtheta=_t(thq), c=_t(c))
    gc_ref = oh.position_vjp(theta, thq, pos, z, f.box, 5.0, None, c)
    e1, e2 = rms_rel(host(g), g_ref), rms_rel(host(gc), gc_ref)
    print("position_vjp", f"{e1:.2e}", f"{e2:.2e}", flush=True)
    assert e1 <= RMS_REL_TOL and e2 <= RMS_REL_TOL


def _training_case(seed):
    f = synth.molten_box(24, seed, L=13.0)
    pol = np.where(f.q > 0, 0.15, 3.5)
    mesh, p, alpha, rc = (16, 16, 16), 6, 0.35, 6.0
    pos, z, a = f32(f.pos), f32(f.q), f32(pol)
    # the teacher on displaced positions, so the student is far from it
    pos_t = f32(pos + np.random.default_rng(seed).normal(scale=0.05, size=pos.shape))
    mu_t = opol.induced_dipoles(pos_t, z, f.box, mesh, p, alpha, rc, a)
    U_t, dUdr_t, _ = opol.model(pos_t, z, mu_t, f.box, mesh, p, alpha, rc, a)
    return f, (mesh, p, alpha, rc), pos, z, a, {"U": U_t, "dUdr": dUdr_t, "mu": mu_t}


@pytest.mark.parametrize("conservative,charge_head",
                         [(True, True), (False, True), (True, False)])
def test_training_gradient_parity(conservative, charge_head):
    """Loss and parameter gradients of one training step (heads -> PME model ->
    conservative or Hellmann-Feynman forces -> loss -> Hessian rows and tangents
    -> both networks) against the oracle."""
    from paper_2606_01598_amd.dip import DipPlan, Trainer
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f, (mesh, p, alpha, rc), pos, z, a, teacher = _training_case(34)
    theta, thq = _params(11)
    kw = dict(lE=1.0, lF=1.0, lmu=0.5, conservative=conservative)
    thq_ref = thq if charge_head else np.zeros(oh.NQPARAM)
    L_ref, g_ref, gq_ref = oh.loss_and_grad(theta, thq_ref, pos, z, a, f.box, mesh, p, alpha, rc,
                                            teacher, **kw)
    x, V = odip.features(pos, z, f.box, 5.0)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pme = Plan(mesh, p, alpha, max_atoms=f.n, keep_phi=True)
    polp = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    dip = DipPlan(f.box, f.n, cutoff=5.0)
    tr = Trainer(dip, polp, pme, box, theta, lr=0.0, lE=1.0, lF=1.0, lmu=0.5,
                 qtheta0=thq if charge_head else None, conservative=conservative)
    b = {"pos": _t(pos), "q": _t(z), "pol": _t(a), "feat": _t(x), "vec": _t(V),
         "U": torch.tensor([teacher["U"]], dtype=torch.float64, device=dev()),
         "dUdr": _t(teacher["dUdr"]), "mu": _t(teacher["mu"])}
    print(f"case: training step conservative={conservative} charge_head={charge_head}",
          flush=True)
    loss = float(host(tr.step(b))[0])
    e_L, e_g = rel(loss, L_ref), rms_rel(host(tr.g), g_ref)
    e_q = rms_rel(host(tr.gq), gq_ref) if charge_head else 0.0
    print("train-grad", conservative, charge_head, f"L {e_L:.2e} g {e_g:.2e} gq {e_q:.2e}",
          flush=True)
    assert e_L <= 1e-4 and e_g <= RMS_REL_TOL and e_q <= RMS_REL_TOL
    # the evaluation call gives the forces the loss used
    ev = tr.evaluate(b)
    F_ref = oh.student(theta, thq_ref, pos, z, a, f.box, mesh, p, alpha, rc,
                       conservative=conservative)["F"]
    e_F = rms_rel(-host(ev["dU_dpos"]), F_ref)
    print("forces", f"{e_F:.2e}", flush=True)
    assert e_F <= RMS_REL_TOL


def test_empty_calls():
    plan = _plan(8)
    theta, thq = _params(12)
    e = torch.empty(0, device=dev())
    e3 = torch.empty(0, 3, device=dev())
    ef = torch.empty(0, odip.NFEAT, device=dev())
    ev = torch.empty(0, odip.NCH, 3, device=dev())
    assert plan.charges(_t(thq), e, ef).numel() == 0
    m, md = plan.forward_jvp(_t(theta), ef, ev, ef, ev)
    assert m.numel() == 0 and md.numel() == 0
    g, gq = plan.backward_jvp(_t(theta), _t(thq), ef, ev, ef, ev, e3, e3, e3, e, e, e)
    assert torch.all(g == 0) and torch.all(gq == 0)
    fd, vd = plan.features_jvp(e3, e, ev, e3)
    assert fd.numel() == 0 and vd.numel() == 0
