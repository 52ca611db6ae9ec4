"""GPU parity of the polarizable-model calls (include/pol.h) against the FP64
oracle (oracle/pol.py), through the C ABI.

Bar, as for the PME path: relative energy error <= 1e-5 and relative RMS error
<= 1e-4 of every per-atom output.  The induced dipoles of the preconditioned CG
solve are compared with the oracle's dense linear solve.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import E_REL_TOL, RMS_REL_TOL, dev, f32, host, rel, rms_rel
from oracle import pol as opol

pytestmark = pytest.mark.gpu


def _frame(n, L, seed):
    f = synth.molten_box(n, seed, L=L)
    pol = np.where(f.q > 0, 0.15, 3.5)
    return f, pol


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev())


def test_real_space_parity():
    from paper_2606_01598_amd.pol import PolPlan
    f, pol = _frame(200, 15.0, 21)
    alpha, rc = 0.35, 6.5
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    out = plan.real(_t(f.pos), _t(f.q), _t(f.mu), _t(pol))
    e, gpos, gmu = opol.real_space(f32(f.pos), f32(f.q), f32(f.mu), f.box, alpha, rc, f32(pol))
    errs = {"E": rel(float(host(out["energy"])[0]), e), "dE_dpos": rms_rel(host(out["dE_dpos"]), gpos),
            "dE_dmu": rms_rel(host(out["dE_dmu"]), gmu)}
    print("real", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["E"] <= E_REL_TOL
    assert errs["dE_dpos"] <= RMS_REL_TOL and errs["dE_dmu"] <= RMS_REL_TOL
    # charges only, dipoles only
    o2 = plan.real(_t(f.pos), None, _t(f.mu), _t(pol), energy=True, dE_dpos=False)
    e2, _, g2 = opol.real_space(f32(f.pos), None, f32(f.mu), f.box, alpha, rc, f32(pol))
    assert rel(float(host(o2["energy"])[0]), e2) <= E_REL_TOL
    assert rms_rel(host(o2["dE_dmu"]), g2) <= RMS_REL_TOL


def test_real_mixed_parity():
    from paper_2606_01598_amd.pol import PolPlan
    f, pol = _frame(160, 14.0, 22)
    alpha, rc = 0.35, 6.0
    v = np.random.default_rng(3).normal(0, 1, (f.n, 3))
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    g = plan.mixed(_t(f.pos), _t(f.q), _t(f.mu), _t(pol), _t(v))
    ref = opol.real_mixed(f32(f.pos), f32(f.q), f32(f.mu), f.box, alpha, rc, f32(pol), f32(v))
    err = rms_rel(host(g), ref)
    print("mixed", f"{err:.2e}", flush=True)
    assert err <= RMS_REL_TOL


def test_scf_matches_dense_solve():
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f, pol = _frame(24, 13.0, 23)
    alpha, rc, mesh, p = 0.35, 6.0, (16, 16, 16), 6
    pme = Plan(mesh, p, alpha, max_atoms=f.n, keep_phi=True)
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    mu, it, res = plan.scf(pme, _t(f.pos), _t(f.q), _t(pol), box, tol=1e-7, max_iter=200)
    ref = opol.induced_dipoles(f32(f.pos), f32(f.q), f.box, mesh, p, alpha, rc, f32(pol))
    err = rms_rel(host(mu), ref)
    print("scf", it, f"{res:.2e}", f"{err:.2e}", flush=True)
    assert res < 1e-7 and it > 0
    assert err <= RMS_REL_TOL
    # warm start from the solution converges at once
    plan_w = PolPlan(f.box, alpha, rc, max_atoms=f.n, warm_start=True)
    mu2 = mu.clone()
    _, it2, res2 = plan_w.scf(pme, _t(f.pos), _t(f.q), _t(pol), box, tol=1e-6, max_iter=200, mu=mu2)
    assert it2 <= 2 and res2 < 1e-6


def test_scf_4096_ions_self_consistent():
    """The 4096-ion teacher box (L = 50.4 A, mesh 50^3, p = 6, r_c = 10 A): the
    solve converges to 1e-6 e*A, and its dipoles zero the gradient of U computed
    by the forward calls (pme_forward + pol_real), independently of the
    Hessian products that the solver used."""
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f = synth.molten_box(4096, 1000)
    pol = np.where(f.q > 0, 0.15, 3.5)
    alpha, rc, mesh, p = 0.30, 10.0, (50, 50, 50), 6
    pme = Plan(mesh, p, alpha, max_atoms=f.n, keep_phi=True)
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pos, q, a = _t(f.pos), _t(f.q), _t(pol)
    mu, it, res = plan.scf(pme, pos, q, a, box, tol=1e-6, max_iter=300)
    print("scf4096", it, f"{res:.2e}", flush=True)
    assert res < 1e-6
    g_lr = pme.forward(pos, q, mu, box)["dE_dmu"]
    g_re = plan.real(pos, q, mu, a, energy=False, dE_dpos=False)["dE_dmu"]
    grad = g_lr + g_re + mu / a[:, None]
    field = g_lr + g_re
    ratio = float(grad.norm() / field.norm())
    print("stationarity", f"{ratio:.2e}", flush=True)
    assert ratio < 1e-4


def test_teacher_4096_ions_matches_oracle():
    """The teacher (self-consistent dipoles, energy and forces) on the 4096-ion
    teacher box against the FP64 oracle's CG solve written by
    tests/golden/make_scf_fullsize.py: the energy, the RMS dipole, and the dipoles
    and forces of a seeded sample of atoms."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_scf_fullsize as ms
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan, teacher
    f, pos, q, pol = ms.inputs()
    print(f"case: teacher, {ms.N} ions, mesh {ms.MESH}", flush=True)
    pme = Plan(ms.MESH, ms.P, ms.ALPHA, max_atoms=ms.N, keep_phi=True)
    plan = PolPlan(f.box, ms.ALPHA, ms.RC, max_atoms=ms.N)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    out = teacher(plan, pme, _t(pos), _t(q), _t(pol), box, tol=1e-7, max_iter=300)
    E, m_rms, atoms, mu_ref, F_ref = ms.read()
    mu = host(out["mu"])
    ii = torch.tensor(atoms, device=dev())
    errs = {"U": rel(float(host(out["energy"])[0]), E),
            "mu_rms": rel(float(np.sqrt(np.mean(np.sum(mu * mu, axis=1)))), m_rms),
            "mu": rms_rel(mu[atoms], mu_ref),
            "F": rms_rel(-host(out["dU_dpos"][ii]), F_ref)}
    print("teacher4096", out["iters"], f"{out['resid']:.2e}", {k: f"{v:.2e}" for k, v in errs.items()},
          flush=True)
    assert out["resid"] < 1e-7
    assert errs["U"] <= E_REL_TOL and errs["mu_rms"] <= E_REL_TOL
    assert errs["mu"] <= RMS_REL_TOL and errs["F"] <= RMS_REL_TOL


def test_model_energy_and_gradients():
    """pol_model against the oracle's U(mu), dU/dr and dU/dmu at random dipoles."""
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f, pol = _frame(24, 13.0, 24)
    alpha, rc, mesh, p = 0.35, 6.0, (16, 16, 16), 6
    pme = Plan(mesh, p, alpha, max_atoms=f.n)
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    out = plan.model(pme, _t(f.pos), _t(f.q), _t(f.mu), _t(pol), box)
    u, gp, gm = opol.model(f32(f.pos), f32(f.q), f32(f.mu), f.box, mesh, p, alpha, rc, f32(pol))
    errs = {"U": rel(float(host(out["energy"])[0]), u), "dU_dpos": rms_rel(host(out["dU_dpos"]), gp),
            "dU_dmu": rms_rel(host(out["dU_dmu"]), gm)}
    print("model", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["U"] <= E_REL_TOL
    assert errs["dU_dpos"] <= RMS_REL_TOL and errs["dU_dmu"] <= RMS_REL_TOL


def test_fixed_iteration_solve_and_graph_replays():
    """POL_F_FIXED_ITERS: exactly max_iter PCG iterations with no host round trip
    give the converging solve's dipoles; the fixed solve and the model evaluation
    captured into a HIP graph replay to the eager results (three replays, eager
    work and synchronisations between them).  The real-space pair sums follow the
    cell list, whose order within a cell is that of atomic insertions, so the
    comparisons allow FP32 rounding amplified by the iterations (1e-4 RMS)."""
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f, pol = _frame(300, 21.0, 23)
    alpha, rc, mesh = 0.35, 8.0, (24, 24, 24)
    pos, q, a = _t(f.pos), _t(f.q), _t(pol)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pme = Plan(mesh, 6, alpha, max_atoms=f.n)
    plan = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    mu_c, it, res = plan.scf(pme, pos, q, a, box, tol=1e-6, max_iter=100)
    assert res < 1e-6 and it > 0
    k = it + it % 2                        # even: 2 + k binnings per captured solve + model
    pme_f = Plan(mesh, 6, alpha, max_atoms=f.n)
    fixed = PolPlan(f.box, alpha, rc, max_atoms=f.n, fixed_iters=True)
    mu_same = torch.zeros(f.n, 3, dtype=torch.float32, device=dev())
    _, it2, res2 = fixed.scf(pme_f, pos, q, a, box, max_iter=it, mu=mu_same)
    assert it2 == it and res2 == -1.0
    assert rms_rel(host(mu_same), host(mu_c)) <= RMS_REL_TOL
    mu_g = torch.zeros(f.n, 3, dtype=torch.float32, device=dev())

    def solve():
        fixed.scf(pme_f, pos, q, a, box, max_iter=k, mu=mu_g)
        return fixed.model(pme_f, pos, q, mu_g, a, box)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ref = {kk: v.clone() for kk, v in solve().items()}
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = solve()
    for r in range(3):
        for v in out.values():
            v.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for kk in ref:
            if kk == "energy":
                assert rel(float(out[kk][0]), float(ref[kk][0])) <= E_REL_TOL, (r, kk)
            else:
                # dU/dmu vanishes at the solution: measured on the scale of the forces
                floor = float(np.sqrt(np.mean(host(ref["dU_dpos"]) ** 2)))
                assert rms_rel(host(out[kk]), host(ref[kk]), floor=floor) <= RMS_REL_TOL, (r, kk)
        plan.model(pme, pos, q, mu_c, a, box)   # eager work between replays
        torch.cuda.synchronize()
    # the fixed-count dipoles are the converged ones: stationarity of U
    stat = float(torch.sqrt(torch.mean(out["dU_dmu"] ** 2)))
    ref_field = float(torch.sqrt(torch.mean(ref["dU_dpos"] ** 2)))
    print("fixed solve: iterations", it, "graph count", k, "rms dU/dmu", stat, flush=True)
    assert stat <= 1e-4 * max(ref_field, 1e-6) + 1e-5
