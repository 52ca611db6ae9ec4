"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar: relative energy error <= 1e-5 (E_recip and E^lr), and for every per-atom
output ||gpu - oracle||_rms / ||oracle||_rms <= 1e-4 (dE/dr, dE/dq, dE/dmu and
the three Hessian-vector-product outputs).  Inputs are seeded synthetic frames;
the oracle sees the same float32-rounded positions, charges and dipoles.
"""
import math

import numpy as np
import pytest
import torch

import synth
from gpu_util import (E_REL_TOL, RMS_REL_TOL, dev, f32, host, oracle_forward, oracle_hvp, rel,
                      rms_rel, to_dev)
from oracle import pme as opme

pytestmark = pytest.mark.gpu


def _plan(mesh, p, alpha, n, **kw):
    from paper_2606_01598_amd.pme import Plan
    return Plan(mesh, p, alpha, max_atoms=max(1, n), **kw)


def _check_forward(frame, mesh, p, alpha, gamma=1.0, with_q=True, with_mu=True, label="",
                   force_floor=0.0, tile=None):
    plan = _plan(mesh, p, alpha, frame.n, influence_power=gamma, tile=tile)
    pos, q, mu, box = to_dev(frame, with_q, with_mu)
    out = plan.forward(pos, q, mu, box)
    plan.status()
    ref = oracle_forward(frame, mesh, p, alpha, gamma, with_q=with_q, with_mu=with_mu)
    e = host(out["energy"])
    errs = {
        "E_recip": rel(e[0], ref.e_recip),
        "E_lr": rel(e.sum(), ref.energy),
        "dE_dpos": rms_rel(host(out["dE_dpos"]), ref.dE_dpos, force_floor),
    }
    if with_q:
        errs["dE_dq"] = rms_rel(host(out["dE_dq"]), ref.dE_dq)
    if with_mu:
        errs["dE_dmu"] = rms_rel(host(out["dE_dmu"]), ref.dE_dmu)
    print(label, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["E_recip"] <= E_REL_TOL and errs["E_lr"] <= E_REL_TOL
    for k in ("dE_dpos", "dE_dq", "dE_dmu"):
        if k in errs:
            assert errs[k] <= RMS_REL_TOL, (k, errs[k])
    assert rel(e[1], ref.e_self_q) < 1e-12 or (not with_q)
    return plan, out, ref


def test_density_and_potential_config1():
    f = synth.rocksalt()
    # the tile spread stores the density; the fused plane spread keeps none
    plan = _plan((16, 16, 16), 4, 0.3, f.n, separate_spread=True)
    pos, q, mu, box = to_dev(f)
    plan.forward(pos, q, mu, box)
    fused = _plan((16, 16, 16), 4, 0.3, f.n)
    fused.forward(pos, q, mu, box)
    with pytest.raises(RuntimeError):
        fused.rho()
    assert torch.equal(fused.phi(), plan.phi())
    ref = oracle_forward(f, (16, 16, 16), 4, 0.3)
    rho, phi = host(plan.rho()), host(plan.phi())
    print("rho", np.abs(rho - ref.rho).max(), "phi", rms_rel(phi, ref.phi), flush=True)
    assert np.abs(rho - ref.rho).max() <= 1e-6 * np.abs(ref.rho).max()
    assert rms_rel(phi, ref.phi) <= 1e-5


def test_forward_config1_rocksalt_charges():
    # 64 ions, p = 4, mesh 16^3, alpha = 0.30
    _check_forward(synth.rocksalt(), (16, 16, 16), 4, 0.3, with_mu=False, label="cfg1")


def test_forward_config2_molten_charges_dipoles():
    f = synth.molten_box(1000, 1, L=31.5)
    _check_forward(f, (32, 32, 32), 6, 0.3, label="cfg2")


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
def test_forward_all_orders_ragged_mesh(p):
    # non-cubic mesh with odd factors: tiles and FFT radices 2, 3, 4, 5 all ragged
    # (the tile target is given, so it is rounded to the bins, 8 x 8 x 15, and not
    # to the dividing tiles of the default, 10 x 10 x 25)
    f = synth.molten_box(300, 10 + p, L=20.0)
    _check_forward(f, (18, 20, 25), p, 0.35, label=f"p{p}", tile=(8, 8, 16))
    if p == 6:
        _check_forward(f, (18, 20, 25), p, 0.35, label=f"p{p} default tiles")


@pytest.mark.parametrize("mesh,p", [((4, 4, 4), 6), ((2, 3, 5), 4), ((6, 6, 6), 7), ((45, 27, 16), 5),
                                    ((64, 50, 30), 6)])
def test_forward_small_and_odd_meshes(mesh, p):
    f = synth.molten_box(120, 21, L=15.0)
    _check_forward(f, mesh, p, 0.4, label=f"mesh{mesh}")


def _random_frame(n, box, seed):
    rng = np.random.default_rng(seed)
    frac = rng.uniform(0, 1, (n, 3))
    q = rng.normal(0, 1, n)
    q -= q.mean()
    return synth.Frame(pos=frac @ box, q=q, mu=rng.normal(0, 0.1, (n, 3)), box=box)


@pytest.mark.parametrize("mesh,p,a", [((32, 32, 32), 6, 0.3), ((12, 160, 150), 5, 0.45)])
def test_fft_lines_per_workgroup(mesh, p, a):
    """The FFT lines per workgroup of the x pass (and of the pencil y pass) set in
    the descriptor: every per-atom output equals the default's bit for bit (each
    line is transformed the same way), the energy only regroups its partial sums."""
    box = np.diag([float(mesh[0]), float(mesh[1]) / 2.0, float(mesh[2]) / 2.0])
    f = _random_frame(300, box, 23)
    pos, q, mu, box_t = to_dev(f)
    v = synth.random_cotangents(f.n, 8, scale_r=0.1)
    vr, vq, vm = (torch.tensor(x, dtype=torch.float32, device=dev()) for x in v)
    outs = []
    for lines in (None, 1, 5, 40):
        plan = _plan(mesh, p, a, f.n, fft_lines=lines)
        o = plan.forward(pos, q, mu, box_t)
        g = plan.backward(pos, q, mu, box_t, vr, vq, vm)
        plan.status()
        outs.append((o, g))
    ref = oracle_forward(f, mesh, p, a)
    e0 = host(outs[0][0]["energy"])
    # E_recip and the forces: this random frame's total energy nearly cancels
    assert rel(e0[0], ref.e_recip) <= E_REL_TOL
    assert rms_rel(host(outs[0][0]["dE_dpos"]), ref.dE_dpos) <= RMS_REL_TOL
    for o, g in outs[1:]:
        for k in ("dE_dpos", "dE_dq", "dE_dmu"):
            assert torch.equal(o[k], outs[0][0][k]), k
        for k in ("g_pos", "g_q", "g_mu"):
            assert torch.equal(g[k], outs[0][1][k]), k
        assert rel(host(o["energy"]).sum(), e0.sum()) <= 1e-12


def test_pencil_mode_mesh_forward_and_hvp():
    # a y-z half-spectrum plane too large for LDS: five pencil passes instead of slabs
    box = np.diag([12.0, 80.0, 75.0])
    f = _random_frame(400, box, 17)
    mesh, p, a = (12, 160, 150), 5, 0.45
    _check_forward(f, mesh, p, a, label="pencil")
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box_t = to_dev(f)
    plan.forward(pos, q, mu, box_t)
    v = synth.random_cotangents(f.n, 3, scale_r=0.1)
    vt = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in v]
    out = plan.backward(pos, q, mu, box_t, *vt)
    ref = oracle_hvp(f, mesh, p, a, v)
    errs = [rms_rel(host(out[k]), r) for k, r in zip(("g_pos", "g_q", "g_mu"), ref)]
    print("pencil hvp", [f"{e:.2e}" for e in errs], flush=True)
    assert max(errs) <= RMS_REL_TOL


def test_forward_triclinic_cell():
    f = synth.triclinic_cell(n=40)
    _check_forward(f, (20, 18, 24), 6, 0.45, label="triclinic")


def test_forward_gamma0_and_prefactor():
    f = synth.molten_box(200, 3, L=18.0)
    _check_forward(f, (20, 20, 20), 5, 0.35, gamma=0.0, label="gamma0")
    plan = _plan((20, 20, 20), 5, 0.35, f.n, prefactor=14.3996454784)
    pos, q, mu, box = to_dev(f)
    out = plan.forward(pos, q, mu, box)
    ref = oracle_forward(f, (20, 20, 20), 5, 0.35, prefactor=14.3996454784)
    assert rel(host(out["energy"]).sum(), ref.energy) <= E_REL_TOL
    assert rms_rel(host(out["dE_dpos"]), ref.dE_dpos) <= RMS_REL_TOL


def test_positions_outside_the_cell():
    f = synth.molten_box(200, 5, L=18.0)
    g = synth.Frame(pos=f.pos + np.array([3, -2, 5]) * 18.0 + 0.0, q=f.q, mu=f.mu, box=f.box)
    _check_forward(g, (20, 20, 20), 6, 0.35, label="images")


def test_empty_and_single_atom():
    plan = _plan((16, 16, 16), 6, 0.3, 4)
    box = torch.eye(3, dtype=torch.float64, device=dev()) * 12.0
    z = torch.zeros(0, 3, dtype=torch.float32, device=dev())
    out = plan.forward(z, torch.zeros(0, device=dev()), z.clone(), box)
    plan.status()
    assert np.all(host(out["energy"]) == 0.0)
    one = synth.Frame(pos=np.array([[1.0, 2.0, 3.0]]), q=np.array([0.7]),
                      mu=np.array([[0.1, -0.2, 0.3]]), box=np.eye(3) * 12.0)
    # the exact force on a lone atom is only the mesh self-force (~5e-7 here):
    # measure the error against the force scale q^2 alpha^2 instead
    _check_forward(one, (16, 16, 16), 6, 0.3, label="one", force_floor=0.7 ** 2 * 0.3 ** 2)


def test_hvp_config2():
    f = synth.molten_box(1000, 1, L=31.5)
    mesh, p, a = (32, 32, 32), 6, 0.3
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    plan.forward(pos, q, mu, box)
    v = synth.random_cotangents(f.n, 5, scale_r=0.1)
    vt = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in v]
    out = plan.backward(pos, q, mu, box, *vt)
    ref = oracle_hvp(f, mesh, p, a, v)
    errs = [rms_rel(host(out[k]), r) for k, r in zip(("g_pos", "g_q", "g_mu"), ref)]
    print("hvp", [f"{e:.2e}" for e in errs], flush=True)
    assert max(errs) <= RMS_REL_TOL


@pytest.mark.parametrize("p,mesh", [(4, (18, 20, 25)), (5, (16, 16, 16)), (7, (20, 20, 20))])
def test_hvp_orders_and_recompute(p, mesh):
    f = synth.molten_box(200, 30 + p, L=17.0)
    v = synth.random_cotangents(f.n, p, scale_r=0.2, scale_mu=0.5)
    ref = oracle_hvp(f, mesh, p, 0.4, v)
    vt = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in v]
    for keep in (True, False):
        plan = _plan(mesh, p, 0.4, f.n, keep_phi=keep)
        pos, q, mu, box = to_dev(f)
        if keep:
            plan.forward(pos, q, mu, box)
        out = plan.backward(pos, q, mu, box, *vt)
        errs = [rms_rel(host(out[k]), r) for k, r in zip(("g_pos", "g_q", "g_mu"), ref)]
        print("hvp", p, keep, [f"{e:.2e}" for e in errs], flush=True)
        assert max(errs) <= RMS_REL_TOL


def test_force_loss_double_backward_through_autograd():
    from paper_2606_01598_amd.pme import pme_energy
    f = synth.molten_box(400, 8, L=23.0)
    mesh, p, a = (24, 24, 24), 6, 0.35
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    q.requires_grad_(True)
    mu.requires_grad_(True)
    pos.requires_grad_(True)
    E = pme_energy(pos, q, mu, box, plan)
    F = -torch.autograd.grad(E, pos, create_graph=True)[0]
    Fref = torch.tensor(np.random.default_rng(2).normal(0, 0.05, (f.n, 3)), dtype=torch.float32,
                        device=dev())
    loss = ((F - Fref) ** 2).mean()
    gq, gmu = torch.autograd.grad(loss, (q, mu))
    # oracle: dL/dF = 2 (F - Fref)/(3N); v_r = -dL/dF; the (q, mu) parts of H v_r
    ref = oracle_forward(f, mesh, p, a)
    vr = -2.0 * (-ref.dE_dpos - f32(host(Fref))) / (3 * f.n)
    hq = opme.hvp(f32(f.pos), f32(f.q), f32(f.mu), f.box, mesh, p, a, v_pos=vr)
    e1, e2 = rms_rel(host(gq), hq[1]), rms_rel(host(gmu), hq[2])
    print("force-loss grads", e1, e2, flush=True)
    assert e1 <= RMS_REL_TOL and e2 <= RMS_REL_TOL


def test_force_loss_two_frames_one_plan():
    """The batch loss of Sec. 2.4 (Eq. loss) sums over frames: two frames through
    one plan, forces of E1 + E2 with create_graph, one force loss, backward.  The
    plan keeps the potential of the second frame only, so the first frame's
    Hessian-vector product must recompute its own.  Every gradient of every frame
    is compared with the oracle's H v (v_r = -dL/dF, v_q = v_mu = 0)."""
    from paper_2606_01598_amd.pme import pme_energy
    mesh, p, a = (24, 24, 24), 6, 0.35
    frames = [synth.molten_box(400, 8, L=23.0), synth.molten_box(400, 9, L=23.0)]
    plan = _plan(mesh, p, a, 400)
    leaves, forces, targets = [], [], []
    E = 0.0
    for k, f in enumerate(frames):
        pos, q, mu, box = to_dev(f)
        for t in (pos, q, mu):
            t.requires_grad_(True)
        leaves.append((pos, q, mu))
        E = E + pme_energy(pos, q, mu, box, plan)
        targets.append(torch.tensor(np.random.default_rng(20 + k).normal(0, 0.05, (f.n, 3)),
                                    dtype=torch.float32, device=dev()))
    grads = torch.autograd.grad(E, [lv[0] for lv in leaves], create_graph=True)
    loss = sum(((-g - t) ** 2).sum() for g, t in zip(grads, targets))
    loss.backward()
    for k, f in enumerate(frames):
        ref = oracle_forward(f, mesh, p, a)
        # dL/dF = 2 (F - Fref), F = -dE/dr: the cotangent on dE/dr is -dL/dF
        vr = -2.0 * (-ref.dE_dpos - f32(host(targets[k])))
        h = opme.hvp(f32(f.pos), f32(f.q), f32(f.mu), f.box, mesh, p, a, v_pos=vr)
        pos, q, mu = leaves[k]
        errs = [rms_rel(host(pos.grad), h[0]), rms_rel(host(q.grad), h[1]),
                rms_rel(host(mu.grad), h[2])]
        print("frame", k, "force-loss H v", [f"{e:.2e}" for e in errs], flush=True)
        assert max(errs) <= RMS_REL_TOL, (k, errs)


def test_phi_id_follows_evaluations():
    """pme_plan_phi_id names the evaluation whose potential is kept; dropping it
    makes the backward recompute (and keep) phi of its own inputs."""
    f = synth.molten_box(200, 31, L=17.0)
    g = synth.molten_box(200, 32, L=17.0)
    mesh, p, a = (16, 16, 16), 6, 0.4
    plan = _plan(mesh, p, a, f.n)
    assert plan.phi_id() == 0
    pf = to_dev(f)
    pg = to_dev(g)
    plan.forward(*pf)
    i1 = plan.phi_id()
    plan.forward(*pg)
    i2 = plan.phi_id()
    assert i1 > 0 and i2 > i1
    v = synth.random_cotangents(f.n, 3, scale_r=0.1)
    vt = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in v]
    plan.drop_phi()
    assert plan.phi_id() == 0
    out = plan.backward(*pf, *vt)
    assert plan.phi_id() > i2
    ref = oracle_hvp(f, mesh, p, a, v)
    errs = [rms_rel(host(out[k]), r) for k, r in zip(("g_pos", "g_q", "g_mu"), ref)]
    assert max(errs) <= RMS_REL_TOL, errs


def test_finite_differences_config2():
    """FP32 GPU gradients against central differences of the GPU energy."""
    f = synth.molten_box(1000, 1, L=31.5)
    mesh, p, a = (32, 32, 32), 6, 0.3
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    out = plan.forward(pos, q, mu, box)
    E = lambda P, Q, M: float(host(plan.forward(P, Q, M, box, dE_dpos=False, dE_dq=False,
                                                  dE_dmu=False)["energy"]).sum())
    rng = np.random.default_rng(3)
    # along q and mu the energy is quadratic: a large step is exact up to rounding
    dq = torch.tensor(rng.normal(0, 0.5, f.n), dtype=torch.float32, device=dev())
    dm = torch.tensor(rng.normal(0, 0.05, (f.n, 3)), dtype=torch.float32, device=dev())
    fdq = (E(pos, q + dq, mu) - E(pos, q - dq, mu)) / 2
    fdm = (E(pos, q, mu + dm) - E(pos, q, mu - dm)) / 2
    assert rel(fdq, float((out["dE_dq"] * dq).sum())) < 1e-3
    assert rel(fdm, float((out["dE_dmu"] * dm).sum())) < 1e-3
    d = torch.tensor(rng.normal(0, 1, (f.n, 3)), dtype=torch.float32, device=dev())
    d /= d.norm()
    # along r: the directional derivative along the step the float32 positions
    # actually take, against central differences of the FP32 energy.  Those carry
    # about 1e-8 relative noise (E_recip ~ 1e3 here, the derivative along a unit
    # global step ~ 0.04), so the sweep also holds a 0.3 A global step (0.005 A per
    # atom), where the oracle's own truncation error is below 1e-4.
    errs = []
    for h in (3e-1, 1e-1, 3e-2, 1e-2, 3e-3):
        pp, pm = pos + h * d, pos - h * d
        an = float((out["dE_dpos"] * (pp - pm)).sum()) / 2
        errs.append(rel((E(pp, q, mu) - E(pm, q, mu)) / 2, an))
    best = min(errs)
    print("fd r", [f"{e:.2e}" for e in errs], flush=True)
    assert best < 1e-3


def test_capacity_and_nonfinite_errors():
    from paper_2606_01598_amd import _lib
    f = synth.molten_box(100, 4, L=15.0)
    plan = _plan((16, 16, 16), 6, 0.3, 50)
    pos, q, mu, box = to_dev(f)
    with pytest.raises(_lib.PMEError) as ei:
        plan.forward(pos, q, mu, box)
    assert ei.value.code == _lib.PME_ECAPACITY
    plan2 = _plan((16, 16, 16), 6, 0.3, f.n)
    bad = pos.clone()
    bad[7, 1] = float("nan")
    plan2.forward(bad, q, mu, box)
    with pytest.raises(_lib.PMEError) as ei:
        plan2.status()
    assert ei.value.code == _lib.PME_ENONFINITE
    # the flag clears and a good call succeeds afterwards
    plan2.forward(pos, q, mu, box)
    plan2.status()


def test_overflowing_bins_still_exact():
    # all atoms crowded into a few mesh cells: bins overflow into the list
    rng = np.random.default_rng(9)
    n = 300
    pos = 5.0 + rng.uniform(0, 1.5, (n, 3))
    q = rng.normal(0, 1, n)
    q -= q.mean()
    f = synth.Frame(pos=pos, q=q, mu=rng.normal(0, 0.1, (n, 3)), box=np.eye(3) * 16.0)
    _check_forward(f, (16, 16, 16), 6, 0.3, label="crowded")


@pytest.mark.parametrize("lo,hi,max_atoms", [((0.2, 0.2, 0.2), (3.8, 3.8, 15.8), 10000),
                                              ((4.0, 4.0, 4.0), (5.5, 5.5, 5.5), 300)])
def test_crowded_tile_hvp_and_step(lo, hi, max_atoms):
    """More atoms in one tile than a gather queues at once (128): 300 atoms in one
    column of 4 bins (64 slots each) of a 16^3 mesh, which fill the tile's first
    round of 256 own slots, and 300 atoms in a 1.5 A cube of a plan with 18 slots
    per bin, most of them in the overflow list; the forward outputs, H v and the
    concurrent pme_step against the oracle."""
    rng = np.random.default_rng(17)
    n = 300
    pos = rng.uniform(lo, hi, (n, 3))
    q = rng.normal(0, 1, n)
    q -= q.mean()
    f = synth.Frame(pos=pos, q=q, mu=rng.normal(0, 0.1, (n, 3)), box=np.eye(3) * 16.0)
    mesh, p, a = (16, 16, 16), 6, 0.3
    v = synth.random_cotangents(n, 23, scale_r=0.1)
    vt = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in v]
    pos_t, q_t, mu_t, box = to_dev(f)
    plan = _plan(mesh, p, a, max_atoms)
    fo = plan.forward(pos_t, q_t, mu_t, box)
    bo = plan.backward(pos_t, q_t, mu_t, box, *vt)
    plan.status()
    ref = oracle_forward(f, mesh, p, a)
    gp, gq, gm = oracle_hvp(f, mesh, p, a, v)
    errs = {"E_lr": rel(host(fo["energy"]).sum(), ref.energy),
            "dE_dpos": rms_rel(host(fo["dE_dpos"]), ref.dE_dpos),
            "g_pos": rms_rel(host(bo["g_pos"]), gp), "g_q": rms_rel(host(bo["g_q"]), gq),
            "g_mu": rms_rel(host(bo["g_mu"]), gm)}
    print("crowded", max_atoms, {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    assert errs["E_lr"] <= E_REL_TOL
    assert max(e for k, e in errs.items() if k != "E_lr") <= RMS_REL_TOL
    cplan = _plan(mesh, p, a, max_atoms, concurrent=True)
    out = cplan.step(pos_t, q_t, mu_t, box, *vt)
    cplan.status()
    want = {**fo, **bo}
    worst = max(float((out[k] - want[k]).abs().max() / want[k].abs().max()) for k in want)
    print("crowded step", max_atoms, f"{worst:.2e}", flush=True)
    assert worst <= 1e-6


def test_config3_32k_full_parity():
    """The 32k-ion, 100^3, p = 6 workload timed by the benchmark, in the same launch
    configuration, against the oracle on every atom."""
    f = synth.molten_box(32000, 3)
    _check_forward(f, (100, 100, 100), 6, 0.3, label="32k")


@pytest.mark.parametrize("mesh,separate,fused", [((32, 32, 32), True, False),
                                                  ((32, 32, 32), False, True),
                                                  ((12, 160, 150), False, False)])
def test_launch_timer_counts_and_outputs_unchanged(mesh, separate, fused):
    """pme_plan_timer brackets exactly the launches of the chosen kind and leaves
    the results untouched, in the slab layout (32^3: one launch per transform half;
    with the fused plane spread, none for the forward half, which the spread
    performs) and the pencil layout (12 x 160 x 150: two launches per transform
    half, the z and y passes; the x pass is one)."""
    from paper_2606_01598_amd import _lib
    f = synth.molten_box(1000, 1)
    plan = _plan(mesh, 6, 0.3, f.n, separate_spread=separate)
    pos, q, mu, box = to_dev(f)
    v = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in
         synth.random_cotangents(f.n, 5, scale_r=0.1)]
    ref = plan.forward(pos, q, mu, box)
    ref_b = plan.backward(pos, q, mu, box, *v)
    per_step = {"bin": 1, "bin_tangent": 1, "spread": 1, "spread_tangent": 1,
                "fft_r2c": 0 if fused else 2, "fft_x": 2, "fft_c2r": 2, "gather": 1, "gather_hvp": 1}
    for kind in _lib.KERNEL_KINDS:
        plan.timer(kind)
        for _ in range(3):
            out = plan.forward(pos, q, mu, box)
            outb = plan.backward(pos, q, mu, box, *v)
        launches, ms = plan.timer_read()
        assert launches == 3 * per_step[kind], (kind, launches)
        assert (0.0 < ms < 1e3) if launches else ms == 0.0, (kind, ms)
        for k in ("dE_dpos", "dE_dq", "dE_dmu"):
            assert torch.equal(out[k], ref[k])
        for k in ("g_pos", "g_q", "g_mu"):
            assert torch.equal(outb[k], ref_b[k])
    plan.timer(None)
    plan.forward(pos, q, mu, box)
    assert plan.timer_read() == (0, 0.0)
    assert plan._lib.pme_plan_timer(plan.handle, _lib.PME_EINVAL + 100) == _lib.PME_EINVAL
    plan.status()


@pytest.mark.parametrize("concurrent", [False, True])
def test_step_equals_forward_then_backward(concurrent):
    """pme_step (forward and H v in one call; with PME_F_CONCURRENT the cotangent
    chain runs on the plan's second stream) gives the outputs of pme_forward
    followed by pme_backward, over several calls in a row (both counter sets of
    each chain), interleaved with plain forward/backward calls, and matches the
    oracle."""
    f = synth.molten_box(3000, 12)   # L = 45.4 A
    mesh, p, a = (48, 45, 50), 6, 0.32
    pos, q, mu, box = to_dev(f)
    v = synth.random_cotangents(f.n, 13, scale_r=0.1)
    vr, vq, vm = (torch.tensor(x, dtype=torch.float32, device=dev()) for x in v)
    ref_plan = _plan(mesh, p, a, f.n)
    fo = ref_plan.forward(pos, q, mu, box)
    bo = ref_plan.backward(pos, q, mu, box, vr, vq, vm)
    plan = _plan(mesh, p, a, f.n, concurrent=concurrent)
    keys = ("energy", "dE_dpos", "dE_dq", "dE_dmu", "g_pos", "g_q", "g_mu")
    want = {**fo, **bo}
    for call in range(3):
        out = plan.step(pos, q, mu, box, vr, vq, vm)
        plan.status()
        worst = max(float((out[k] - want[k]).abs().max() / want[k].abs().max()) for k in keys)
        print("step", concurrent, call, f"{worst:.2e}", flush=True)
        assert worst <= 1e-6
        # a plain forward/backward between steps keeps both paths consistent
        fo2 = plan.forward(pos, q, mu, box)
        bo2 = plan.backward(pos, q, mu, box, vr, vq, vm)
        assert float((bo2["g_pos"] - bo["g_pos"]).abs().max() / bo["g_pos"].abs().max()) <= 1e-6
        assert float((fo2["dE_dpos"] - fo["dE_dpos"]).abs().max() / fo["dE_dpos"].abs().max()) <= 1e-6
    ref = oracle_forward(f, mesh, p, a)
    assert rel(host(out["energy"]).sum(), ref.energy) <= E_REL_TOL
    assert rms_rel(host(out["dE_dpos"]), ref.dE_dpos) <= RMS_REL_TOL
    gp, gq, gm = oracle_hvp(f, mesh, p, a, (host(vr), host(vq), host(vm)))
    assert rms_rel(host(out["g_pos"]), gp) <= RMS_REL_TOL
    assert rms_rel(host(out["g_q"]), gq) <= RMS_REL_TOL
    assert rms_rel(host(out["g_mu"]), gm) <= RMS_REL_TOL


def test_step_edge_cases_concurrent():
    """pme_step with PME_F_CONCURRENT: no atoms; a pencil-layout mesh with odd
    sizes; cotangents on positions only (the force-loss case, v_q = v_mu = NULL),
    each against pme_forward + pme_backward of a plain plan."""
    # no atoms: zero energy, nothing written
    plan = _plan((16, 16, 16), 6, 0.3, 4, concurrent=True)
    box = torch.eye(3, dtype=torch.float64, device=dev()) * 12.0
    z = torch.zeros(0, 3, dtype=torch.float32, device=dev())
    out = plan.step(z, torch.zeros(0, device=dev()), z.clone(), box, z.clone(),
                    torch.zeros(0, device=dev()), z.clone())
    plan.status()
    assert np.all(host(out["energy"]) == 0.0)
    # pencil layout, odd sizes, position-only cotangents
    box_np = np.diag([12.0, 80.0, 75.0])
    f = _random_frame(400, box_np, 21)
    mesh, p, a = (12, 160, 150), 5, 0.45
    pos, q, mu, box_t = to_dev(f)
    vr = torch.tensor(synth.random_cotangents(f.n, 4, scale_r=0.1)[0], dtype=torch.float32,
                      device=dev())
    ref_plan = _plan(mesh, p, a, f.n)
    want = {**ref_plan.forward(pos, q, mu, box_t), **ref_plan.backward(pos, q, mu, box_t, vr)}
    plan = _plan(mesh, p, a, f.n, concurrent=True)
    for call in range(2):
        out = plan.step(pos, q, mu, box_t, vr)
        plan.status()
        worst = max(float((out[k] - want[k]).abs().max() / want[k].abs().max()) for k in want)
        print("step pencil", call, f"{worst:.2e}", flush=True)
        assert worst <= 1e-6
