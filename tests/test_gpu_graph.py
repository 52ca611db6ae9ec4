"""The captured step graph (pme_step_capture / pme_step_replay, through the C ABI):
every replay, with eager calls on the plan between replays, gives the eager
pme_step outputs bit for bit (the spread is exact fixed point and every reduction
has a fixed order); set-parity rules; the launch timer around graph replays."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("energy", "dE_dpos", "dE_dq", "dE_dmu", "g_pos", "g_q", "g_mu")


def _setup(n, seed, L=None, concurrent=True, mesh=(32, 32, 32), p=6, alpha=0.3):
    from paper_2606_01598_amd.pme import Plan
    f = synth.molten_box(n, seed, L=L)
    pos, q, mu, box = to_dev(f)
    v = [torch.tensor(x, dtype=torch.float32, device=dev())
         for x in synth.random_cotangents(n, seed + 50, scale_r=0.1)]
    plan = Plan(mesh, p, alpha, max_atoms=n, concurrent=concurrent)
    return plan, (pos, q, mu, box), v


@pytest.mark.parametrize("concurrent,steps", [(True, 2), (True, 4), (False, 1)])
def test_replays_equal_eager_steps(concurrent, steps):
    plan, (pos, q, mu, box), v = _setup(1000, 1, L=31.5, concurrent=concurrent)
    for _ in range(4):
        ref = plan.step(pos, q, mu, box, *v)
    plan.status()
    out = plan.step_capture(steps, pos, q, mu, box, *v)
    for r in range(3):
        for t in out.values():
            t.fill_(float("nan"))
        plan.step_replay()
        plan.status()
        for k in KEYS:
            assert torch.equal(out[k], ref[k]), (r, k)
        # eager work on the plan between replays (parity-neutral)
        for _ in range(2):
            e = plan.step(pos, q, mu, box, *v)
        plan.status()
        for k in KEYS:
            assert torch.equal(e[k], ref[k]), (r, k, "eager")


def test_parity_rules():
    from paper_2606_01598_amd._lib import PME_EINVAL, PMEError
    plan, (pos, q, mu, box), v = _setup(400, 2, L=22.0, mesh=(24, 24, 24))
    ref = plan.step(pos, q, mu, box, *v)
    ref = {k: t.clone() for k, t in plan.step(pos, q, mu, box, *v).items()}
    with pytest.raises(PMEError) as ei:
        plan.step_capture(3, pos, q, mu, box, *v)       # odd: the sets would not alternate back
    assert ei.value.code == PME_EINVAL
    with pytest.raises(PMEError) as ei:
        plan.step_replay()                               # no graph
    assert ei.value.code == PME_EINVAL
    out = plan.step_capture(2, pos, q, mu, box, *v)
    plan.forward(pos, q, mu, box)                        # one binning: parity changed
    with pytest.raises(PMEError) as ei:
        plan.step_replay()
    assert ei.value.code == PME_EINVAL
    plan.forward(pos, q, mu, box)                        # and restored
    plan.step_replay()
    plan.status()
    for k in KEYS:
        assert torch.equal(out[k], ref[k]), k


def test_timer_and_graph():
    """Launches captured into the graph are not timed; eager launches around the
    replays are, as before."""
    plan, (pos, q, mu, box), v = _setup(1000, 3, L=31.5)
    for _ in range(2):
        plan.step(pos, q, mu, box, *v)
    plan.timer("spread_tangent")
    plan.step_capture(4, pos, q, mu, box, *v)
    plan.step_replay()
    k, _ = plan.timer_read()
    assert k == 0
    plan.step(pos, q, mu, box, *v)
    plan.step(pos, q, mu, box, *v)
    plan.step_replay()
    k2, ms2 = plan.timer_read()
    assert k2 == 2 and ms2 > 0.0
    plan.timer(None)
    plan.status()


def test_graph_with_optimal_influence_and_sequential_plan():
    """Replays of a plan with the optimal influence function equal its eager steps."""
    from paper_2606_01598_amd.pme import Plan
    f = synth.molten_box(400, 7, L=22.0)
    pos, q, mu, box = to_dev(f)
    v = [torch.tensor(x, dtype=torch.float32, device=dev())
         for x in synth.random_cotangents(f.n, 57, scale_r=0.1)]
    plan = Plan((24, 24, 24), 5, 0.35, max_atoms=f.n, concurrent=True, optimal_influence=True)
    ref = {k: t.clone() for k, t in plan.step(pos, q, mu, box, *v).items()}
    plan.step(pos, q, mu, box, *v)
    out = plan.step_capture(2, pos, q, mu, box, *v)
    for _ in range(2):
        plan.step_replay()
        plan.status()
        for k in KEYS:
            assert torch.equal(out[k], ref[k]), k



def test_graph_at_the_32k_workload():
    """The benchmark's configuration (32k ions, 100^3, p = 6, concurrent chains):
    replays equal the eager steps bit for bit."""
    plan, (pos, q, mu, box), v = _setup(32000, 3, mesh=(100, 100, 100))
    ref = {k: t.clone() for k, t in plan.step(pos, q, mu, box, *v).items()}
    plan.step(pos, q, mu, box, *v)
    out = plan.step_capture(4, pos, q, mu, box, *v)
    for _ in range(2):
        for t in out.values():
            t.fill_(float("nan"))
        plan.step_replay()
        plan.status()
        for k in KEYS:
            assert torch.equal(out[k], ref[k]), k
