"""GPU parity of the optimal influence function (plan flag PME_F_OPT_INFLUENCE,
through the C ABI) against the FP64 oracle with the same influence: forward
outputs and the Hessian-vector product, on a fine and on a coarse mesh (where the
aliasing sums matter), a triclinic cell and the pencil layout; pme_step with it;
the combinations the library rejects.

Bar: as for the deconvolution (relative energy error <= 1e-5, per-atom outputs
<= 1e-4 in RMS).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import (E_REL_TOL, RMS_REL_TOL, dev, host, oracle_forward, oracle_hvp, rel,
                      rms_rel, to_dev)

pytestmark = pytest.mark.gpu


def _plan(mesh, p, alpha, n, **kw):
    from paper_2606_01598_amd.pme import Plan
    return Plan(mesh, p, alpha, max_atoms=max(n, 1), optimal_influence=True, **kw)


def _check(f, mesh, p, a, label):
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    out = plan.forward(pos, q, mu, box)
    v = synth.random_cotangents(f.n, 7, scale_r=0.1)
    vt = [torch.tensor(x, dtype=torch.float32, device=dev()) for x in v]
    hv = plan.backward(pos, q, mu, box, *vt)
    plan.status()
    ref = oracle_forward(f, mesh, p, a, gamma="optimal")
    gp, gq, gm = oracle_hvp(f, mesh, p, a, v, gamma="optimal")
    e = host(out["energy"])
    errs = {"E_recip": rel(e[0], ref.e_recip), "E_lr": rel(e.sum(), ref.energy),
            "dE_dpos": rms_rel(host(out["dE_dpos"]), ref.dE_dpos),
            "dE_dq": rms_rel(host(out["dE_dq"]), ref.dE_dq),
            "dE_dmu": rms_rel(host(out["dE_dmu"]), ref.dE_dmu),
            "g_pos": rms_rel(host(hv["g_pos"]), gp), "g_q": rms_rel(host(hv["g_q"]), gq),
            "g_mu": rms_rel(host(hv["g_mu"]), gm)}
    print(label, {k: f"{x:.2e}" for k, x in errs.items()}, flush=True)
    assert errs["E_recip"] <= E_REL_TOL and errs["E_lr"] <= E_REL_TOL
    assert max(x for k, x in errs.items() if not k.startswith("E")) <= RMS_REL_TOL
    return plan


def test_optimal_influence_fine_mesh():
    f = synth.molten_box(1000, 1, L=31.5)
    _check(f, (32, 32, 32), 6, 0.3, "fine")


def test_optimal_influence_coarse_mesh():
    f = synth.molten_box(200, 2)
    _check(f, (10, 12, 10), 4, 0.45, "coarse")


def test_optimal_influence_triclinic_and_pencil():
    rng = np.random.default_rng(5)
    n = 300
    box = np.array([[16.0, 0.5, -0.4], [1.2, 15.0, 0.7], [-0.8, 1.1, 17.0]])
    q = rng.normal(0.0, 1.0, n)
    q -= q.mean()
    f = synth.Frame(pos=rng.uniform(0, 1, (n, 3)) @ box, q=q, mu=rng.normal(0, 0.2, (n, 3)),
                    box=box)
    _check(f, (16, 15, 18), 5, 0.4, "triclinic")
    box = np.diag([12.0, 80.0, 75.0])
    f = synth.Frame(pos=rng.uniform(0, 1, (n, 3)) @ box, q=q, mu=rng.normal(0, 0.2, (n, 3)),
                    box=box)
    _check(f, (12, 160, 150), 5, 0.45, "pencil")


def test_optimal_influence_step_and_rejections():
    from paper_2606_01598_amd._lib import PME_EINVAL, PMEError
    f = synth.molten_box(400, 3, L=22.0)
    mesh, p, a = (24, 24, 24), 6, 0.35
    pos, q, mu, box = to_dev(f)
    v = [torch.tensor(x, dtype=torch.float32, device=dev())
         for x in synth.random_cotangents(f.n, 9, scale_r=0.1)]
    ref = _plan(mesh, p, a, f.n)
    want = {**ref.forward(pos, q, mu, box), **ref.backward(pos, q, mu, box, *v)}
    plan = _plan(mesh, p, a, f.n, concurrent=True)
    out = plan.step(pos, q, mu, box, *v)
    plan.status()
    worst = max(float((out[k] - want[k]).abs().max() / want[k].abs().max()) for k in want)
    assert worst <= 1e-6
    with pytest.raises(PMEError) as ei:
        ref.forward(pos, q, mu, box, cell=True)
    assert ei.value.code == PME_EINVAL


def test_optimal_influence_cache_follows_the_box():
    """g is cached per box: a repeated box reads it (bit-identical outputs), a new
    box recomputes it (parity with the oracle at that box), and returning to the
    first box gives its outputs again."""
    f = synth.molten_box(400, 4, L=22.0)
    mesh, p, a = (24, 24, 24), 5, 0.4
    plan = _plan(mesh, p, a, f.n)
    pos, q, mu, box = to_dev(f)
    o1 = {k: t.clone() for k, t in plan.forward(pos, q, mu, box).items()}
    o2 = plan.forward(pos, q, mu, box)
    for k in o1:
        assert torch.equal(o1[k], o2[k]), k
    box2 = torch.tensor(np.diag([22.5, 21.5, 22.0]), dtype=torch.float64, device=dev())
    o3 = plan.forward(pos, q, mu, box2)
    plan.status()
    g = synth.Frame(pos=f.pos, q=f.q, mu=f.mu, box=np.diag([22.5, 21.5, 22.0]))
    ref = oracle_forward(g, mesh, p, a, gamma="optimal")
    assert rel(host(o3["energy"]).sum(), ref.energy) <= E_REL_TOL
    assert rms_rel(host(o3["dE_dpos"]), ref.dE_dpos) <= RMS_REL_TOL
    o4 = plan.forward(pos, q, mu, box)
    for k in o1:
        assert torch.equal(o1[k], o4[k]), k
