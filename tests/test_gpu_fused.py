"""The spread fused with the forward slab transform (one x-plane per workgroup,
the default where the padded plane fits in LDS) against the tile spread followed by
the separate slab transform (PME_F_SEPARATE_SPREAD): every output of pme_forward,
pme_backward and the concurrent pme_step must be bitwise equal, since both add the
same 64-bit fixed-point contributions and transform the same density.  The cases
cover orders 4-7, odd, ragged and non-cubic meshes, a sheared cell, the benchmark
box, a clustered box whose bins overflow, a dense box whose scanned slots exceed
the item map (binary search), and a crowded box whose planes hold more atoms than
the hit list (drained in batches).  Parity with the oracle of the fused path
itself is checked by the PME tests, which use default plans."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu


def _frame(case):
    if case == "clustered":
        rng = np.random.default_rng(5)
        n, L = 2000, 24.0
        pos = rng.uniform(0.0, 6.0, (n, 3))   # one corner: bins far over capacity
        q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
        return synth.Frame(pos=pos, q=q, mu=rng.normal(0, 0.1, (n, 3)), box=np.eye(3) * L)
    if case == "crowded":
        rng = np.random.default_rng(6)
        n, L = 12000, 24.0
        pos = rng.uniform(0.0, L, (n, 3))
        pos[:, 0] = rng.uniform(0.0, 1.5, n)   # a few x-planes hold every atom
        q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
        return synth.Frame(pos=pos, q=q, mu=rng.normal(0, 0.1, (n, 3)), box=np.eye(3) * L)
    if case == "sheared":
        f = synth.molten_box(1200, 8, L=32.0)
        box = f.box.copy()
        box[1, 0] = 3.0
        box[2, 0] = -2.0
        box[2, 1] = 1.5
        return synth.Frame(pos=f.pos, q=f.q, mu=f.mu, box=box)
    n, seed, L = {"small": (400, 1, 20.0), "ragged": (800, 2, 30.0), "p7": (1500, 3, 36.0),
                  "p4": (300, 4, 22.0), "8k": (8000, 2, None), "32k": (32000, 3, None),
                  "dense": (32000, 3, None)}[case]
    return synth.molten_box(n, seed, L=L)


CASES = [("small", (24, 24, 24), 6), ("ragged", (30, 36, 40), 5), ("p7", (40, 40, 40), 7),
         ("p4", (20, 24, 30), 4), ("sheared", (27, 30, 32), 6), ("clustered", (24, 24, 24), 6),
         ("dense", (48, 48, 48), 6), ("crowded", (24, 24, 24), 6), ("8k", (64, 64, 64), 6),
         ("32k", (100, 100, 100), 6)]


@pytest.mark.parametrize("case,mesh,p", CASES, ids=[c[0] for c in CASES])
def test_fused_spread_equals_tile_spread(case, mesh, p):
    from paper_2606_01598_amd.pme import Plan
    f = _frame(case)
    print(f"case: fused spread {case} n={len(f.q)} mesh={mesh} p={p}", flush=True)
    d = dev()
    t = lambda a, dt=torch.float32: torch.tensor(np.asarray(a), dtype=dt, device=d)
    pos, q, mu, box = t(f.pos), t(f.q), t(f.mu), t(f.box, torch.float64)
    v = [t(x) for x in synth.random_cotangents(len(f.q), 9, scale_r=0.1)]
    alpha = 0.35
    outs = []
    for separate in (False, True):
        plan = Plan(mesh, p, alpha, max_atoms=len(f.q), separate_spread=separate)
        assert plan.spread_kind == ("tile" if separate else "fused"), (case, plan.spread_kind)
        plan.timer("fft_r2c")
        o = {k: x.clone() for k, x in plan.forward(pos, q, mu, box).items()}
        launches, _ = plan.timer_read()
        plan.timer(None)
        assert launches == (1 if separate else 0), (separate, launches)   # fused: no r2c pass
        o.update({k: x.clone() for k, x in plan.backward(pos, q, mu, box, *v).items()})
        step = Plan(mesh, p, alpha, max_atoms=len(f.q), concurrent=True, separate_spread=separate)
        o.update({"step_" + k: x.clone() for k, x in step.step(pos, q, mu, box, *v).items()})
        plan.status()
        step.status()
        outs.append(o)
    fused, tile = outs
    for k in tile:
        assert torch.equal(fused[k], tile[k]), (case, k)
    assert float(tile["energy"].abs().sum()) > 0.0
