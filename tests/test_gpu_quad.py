"""GPU parity of the quadrupole channel (pme_forward_quad, through the C ABI)
against the FP64 oracle (oracle/quad.py, pinned on the CPU by charge-cluster
limits, rotation invariance, finite differences and the Ewald limit), on the
same float32-rounded inputs.

Bar: relative error of E_recip and E^lr <= 1e-5; ||gpu - oracle||_rms /
||oracle||_rms <= 1e-4 for dE/dr, dE/dq, dE/dmu and dE/dTheta (as for the
charge + dipole forward); the Theta self term, a double sum of float inputs on
both sides, to 1e-9.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import E_REL_TOL, RMS_REL_TOL, dev, f32, host, rel, rms_rel, to_dev
from oracle import quad as oquad

pytestmark = pytest.mark.gpu


def _plan(mesh, p, alpha, n, **kw):
    from paper_2606_01598_amd.pme import Plan
    return Plan(mesh, p, alpha, max_atoms=max(n, 1), **kw)


def _check(frame, th, mesh, p, alpha, label, with_q=True, with_mu=True, prefactor=1.0,
           max_atoms=None, **kw):
    plan = _plan(mesh, p, alpha, max_atoms or frame.n, prefactor=prefactor, **kw)
    pos, q, mu, box = to_dev(frame, with_q, with_mu)
    tht = torch.tensor(th, dtype=torch.float32, device=dev())
    out = plan.forward(pos, q, mu, box, theta=tht)
    plan.status()
    ref = oquad.forward(f32(frame.pos), f32(frame.q) if with_q else None,
                        f32(frame.mu) if with_mu else None, f32(th), frame.box, mesh, p, alpha,
                        prefactor=prefactor, **({"gamma": "optimal"} if kw.get("optimal_influence") else {}))
    e = host(out["energy"])
    errs = {"E_recip": rel(e[0], ref.e_recip), "E_lr": rel(e.sum(), ref.energy),
            "dE_dpos": rms_rel(host(out["dE_dpos"]), ref.dE_dpos),
            "dE_dtheta": rms_rel(host(out["dE_dtheta"]), ref.dE_dtheta)}
    if with_q:
        errs["dE_dq"] = rms_rel(host(out["dE_dq"]), ref.dE_dq)
    if with_mu:
        errs["dE_dmu"] = rms_rel(host(out["dE_dmu"]), ref.dE_dmu)
    print(label, {k: f"{x:.2e}" for k, x in errs.items()}, flush=True)
    assert errs["E_recip"] <= E_REL_TOL and errs["E_lr"] <= E_REL_TOL
    assert max(x for k, x in errs.items() if not k.startswith("E")) <= RMS_REL_TOL
    assert rel(e[3], ref.e_self_theta) <= 1e-9
    return plan, out, ref


def test_quad_molten_box():
    f = synth.molten_box(1000, 1, L=31.5)
    _check(f, synth.random_quadrupoles(f.n, 21), (32, 32, 32), 6, 0.3, "molten 1000 p6")


def test_quad_triclinic_and_prefactor():
    rng = np.random.default_rng(5)
    n = 300
    box = np.array([[16.0, 0.5, -0.4], [1.2, 15.0, 0.7], [-0.8, 1.1, 17.0]])
    q = rng.normal(0.0, 1.0, n)
    q -= q.mean()
    f = synth.Frame(pos=rng.uniform(-1.0, 2.0, (n, 3)) @ box, q=q, mu=rng.normal(0, 0.2, (n, 3)),
                    box=box)
    _check(f, synth.random_quadrupoles(n, 22, scale=0.5), (16, 15, 18), 5, 0.4, "triclinic p5",
           prefactor=14.399645)


def test_quad_pencil_layout_order4():
    rng = np.random.default_rng(17)
    n = 400
    box = np.diag([12.0, 80.0, 75.0])
    q = rng.normal(0.0, 1.0, n)
    q -= q.mean()
    f = synth.Frame(pos=rng.uniform(0.0, 1.0, (n, 3)) @ box, q=q, mu=rng.normal(0, 0.2, (n, 3)),
                    box=box)
    _check(f, synth.random_quadrupoles(n, 23), (12, 160, 150), 4, 0.45, "pencil p4")


@pytest.mark.parametrize("with_q,with_mu", [(False, False), (True, False)])
def test_quad_without_dipoles_order7(with_q, with_mu):
    f = synth.molten_box(500, 6, L=25.0, mu_sigma=0.3)
    _check(f, synth.random_quadrupoles(f.n, 24, traceless=True), (27, 25, 24), 7, 0.32,
           f"p7 q={with_q} mu={with_mu}", with_q, with_mu)


def test_quad_with_optimal_influence():
    f = synth.molten_box(400, 3, L=22.0)
    _check(f, synth.random_quadrupoles(f.n, 25), (16, 16, 16), 5, 0.4, "optimal influence",
           optimal_influence=True)


def test_quad_zero_theta_is_pme_forward():
    f = synth.molten_box(600, 2, L=26.0)
    mesh, p, a = (27, 27, 27), 6, 0.3
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    z = torch.zeros(f.n, 6, dtype=torch.float32, device=dev())
    r = plan.forward(pos, q, mu, box, theta=z)
    s = plan.forward(pos, q, mu, box)
    plan.status()
    assert float(r["energy"][3]) == 0.0
    for k in ("dE_dpos", "dE_dq", "dE_dmu"):
        d = float((r[k] - s[k]).abs().max() / s[k].abs().max())
        assert d <= 1e-5, (k, d)
    assert np.abs(host(r["dE_dtheta"])).max() > 0.0     # the gradient is not zero at 0
    assert abs(float(r["energy"][:3].sum() - s["energy"].sum())) <= 1e-6 * abs(float(s["energy"].sum()))


def test_quad_rejections_and_no_atoms():
    from paper_2606_01598_amd._lib import PME_EINVAL, PMEError
    f = synth.molten_box(100, 4, L=14.0)
    pos, q, mu, box = to_dev(f)
    th = torch.tensor(synth.random_quadrupoles(f.n, 26), dtype=torch.float32, device=dev())
    plan3 = _plan((16, 16, 16), 3, 0.4, f.n)
    with pytest.raises(PMEError) as ei:
        plan3.forward(pos, q, mu, box, theta=th)
    assert ei.value.code == PME_EINVAL
    plan = _plan((16, 16, 16), 5, 0.4, f.n)
    with pytest.raises(ValueError):
        plan.forward(pos, q, mu, box, theta=th, cell=True)
    z3 = torch.zeros(0, 3, dtype=torch.float32, device=dev())
    out = plan.forward(z3, torch.zeros(0, device=dev()), z3.clone(), box,
                       theta=torch.zeros(0, 6, dtype=torch.float32, device=dev()))
    plan.status()
    assert np.all(host(out["energy"]) == 0.0)


def test_quad_32k_workload():
    """The 32k-ion, 100^3, p = 6 workload of the benchmark with second moments."""
    f = synth.molten_box(32000, 3)
    _check(f, synth.random_quadrupoles(f.n, 27), (100, 100, 100), 6, 0.3, "32k")


def test_quad_through_autograd():
    """pme_energy with theta: the gradients autograd returns are those of
    pme_forward_quad, scaled by the upstream gradient."""
    from paper_2606_01598_amd.pme import pme_energy
    f = synth.molten_box(400, 9, L=22.0)
    mesh, p, a = (24, 24, 24), 6, 0.35
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    th = torch.tensor(synth.random_quadrupoles(f.n, 28), dtype=torch.float32, device=dev())
    ref = plan.forward(pos, q, mu, box, theta=th)
    for t in (pos, q, mu, th):
        t.requires_grad_(True)
    e = pme_energy(pos, q, mu, box, plan, theta=th)
    (3.0 * e).backward()
    assert abs(float(e.detach()) - float(ref["energy"].sum())) <= 1e-12 * abs(float(e.detach()))
    for t, k in ((pos, "dE_dpos"), (q, "dE_dq"), (mu, "dE_dmu"), (th, "dE_dtheta")):
        assert torch.allclose(t.grad, 3.0 * ref[k], rtol=1e-6, atol=0.0), k


@pytest.mark.parametrize("lo,hi,max_atoms", [((0.2, 0.2, 0.2), (3.8, 3.8, 15.8), 10000),
                                             ((4.0, 4.0, 4.0), (5.5, 5.5, 5.5), 300)])
def test_quad_crowded_tile(lo, hi, max_atoms):
    """More atoms in one tile than a gather queues at once (a column of 4 bins with
    64 slots each), and 300 atoms in a 1.5 A cube of a plan with 18 slots per bin,
    most of them in the overflow list."""
    rng = np.random.default_rng(18)
    n = 300
    q = rng.normal(0, 1, n)
    q -= q.mean()
    f = synth.Frame(pos=rng.uniform(lo, hi, (n, 3)), q=q, mu=rng.normal(0, 0.1, (n, 3)),
                    box=np.eye(3) * 16.0)
    _check(f, synth.random_quadrupoles(n, 29, scale=0.1), (16, 16, 16), 6, 0.3,
           f"crowded {max_atoms}", max_atoms=max_atoms)
