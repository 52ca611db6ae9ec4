"""The band spread (one workgroup per band of y-rows of an x-plane, the default on
meshes whose padded y-z plane does not fit in LDS beside the slab transform)
against the tile spread (PME_F_SEPARATE_SPREAD): every output of pme_forward,
pme_backward and the concurrent pme_step must be bitwise equal, since both add the
same 64-bit fixed-point contributions to each mesh point.  The cases cover orders
1-7, slab and pencil layouts, bands that do not divide N_y, a sheared cell, a
clustered box whose bins overflow, a crowded box whose bands scan more slots than
the item map holds and list more atoms than the hit list (drained in batches), and
a grid deep enough for the bands sized for two workgroups per CU.  The oracle parity of the band path itself is checked by the PME tests
on these layouts and by the 128k and 1M full-size tests."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu


def _frame(case, diag):
    rng = np.random.default_rng({"plain": 21, "clustered": 22, "crowded": 23, "sheared": 24}[case])
    diag = np.asarray(diag, dtype=float)
    n = {"plain": 3000, "clustered": 3000, "crowded": 20000, "sheared": 3000}[case]
    pos = rng.uniform(0.0, 1.0, (n, 3)) * diag
    if case == "clustered":
        pos = rng.uniform(0.0, 5.0, (n, 3))           # one corner: bins far over capacity
    if case == "crowded":
        pos[:, 0] = rng.uniform(0.0, 1.5, n)           # a few x-planes hold every atom
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    box = np.diag(diag)
    if case == "sheared":
        box[1, 0] = 3.0
        box[2, 0] = -2.0
        box[2, 1] = 1.5
    return synth.Frame(pos=pos, q=q, mu=rng.normal(0.0, 0.1, (n, 3)), box=box)


# mesh, order, box edges (about 1 A per mesh point), frame
CASES = [("slab", (40, 128, 128), 6, (40.0, 128.0, 128.0), "plain"),
         ("pencil", (12, 160, 150), 5, (12.0, 160.0, 150.0), "plain"),
         ("ragged_p7", (36, 125, 135), 7, (36.0, 125.0, 135.0), "plain"),
         ("p4", (32, 150, 120), 4, (32.0, 150.0, 120.0), "sheared"),
         ("clustered", (40, 128, 128), 6, (40.0, 128.0, 128.0), "clustered"),
         ("crowded", (40, 128, 128), 6, (40.0, 128.0, 128.0), "crowded"),
         ("p1", (24, 128, 120), 1, (24.0, 128.0, 120.0), "plain"),
         ("p2", (24, 128, 120), 2, (24.0, 128.0, 120.0), "plain"),
         ("p3", (24, 150, 125), 3, (24.0, 150.0, 125.0), "sheared"),
         # 256 planes of 4 bands: a grid of 1024 workgroups, so bands sized for two
         # workgroups per CU
         ("pair", (256, 200, 200), 6, (256.0, 200.0, 200.0), "plain")]


@pytest.mark.parametrize("case,mesh,p,diag,kind", CASES, ids=[c[0] for c in CASES])
def test_band_spread_equals_tile_spread(case, mesh, p, diag, kind):
    from paper_2606_01598_amd.pme import Plan
    f = _frame(kind, diag)
    n = len(f.q)
    print(f"case: band spread {case} n={n} mesh={mesh} p={p}", flush=True)
    d = dev()
    t = lambda a, dt=torch.float32: torch.tensor(np.asarray(a), dtype=dt, device=d)
    pos, q, mu, box = t(f.pos), t(f.q), t(f.mu), t(f.box, torch.float64)
    v = [t(x) for x in synth.random_cotangents(n, 19, scale_r=0.1)]
    alpha = 0.35
    outs = []
    for separate in (False, True):
        plan = Plan(mesh, p, alpha, max_atoms=n, separate_spread=separate)
        assert plan.spread_kind == ("tile" if separate else "band"), (case, plan.spread_kind)
        o = {k: x.clone() for k, x in plan.forward(pos, q, mu, box).items()}
        o["rho"] = plan.rho()
        o.update({"hvp_" + k: x.clone() for k, x in plan.backward(pos, q, mu, box, *v).items()})
        o["rho_tangent"] = plan.rho()
        step = Plan(mesh, p, alpha, max_atoms=n, concurrent=True, separate_spread=separate)
        o.update({"step_" + k: x.clone() for k, x in step.step(pos, q, mu, box, *v).items()})
        plan.status()
        step.status()
        outs.append(o)
    band, tile = outs
    for k in tile:
        assert torch.equal(band[k], tile[k]), (case, k)
    assert float(tile["energy"].abs().sum()) > 0.0
    assert float(tile["rho"].abs().sum()) > 0.0
