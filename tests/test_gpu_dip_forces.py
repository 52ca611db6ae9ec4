"""GPU parity of the conservative student forces (dip_position_vjp, through the C
ABI) against the FP64 oracle (oracle/dip.py: position_vjp, conservative_forces,
pinned on the CPU by finite differences of the dipoles and of the total model
energy).

Bar: relative RMS error <= 1e-4 (as for the rest of the dipole head).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import RMS_REL_TOL, dev, f32, host, rms_rel
from oracle import dip as odip

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev())


@pytest.mark.parametrize("n,seed,L", [(300, 31, None), (600, 34, None), (40, 35, 12.0)])
def test_position_vjp_parity(n, seed, L):
    from paper_2606_01598_amd.dip import DipPlan
    f = synth.molten_box(n, seed, L=L)
    plan = DipPlan(f.box, f.n, cutoff=5.0)
    pos, q = _t(f.pos), _t(f.q)
    feat, vec = plan.features(pos, q)
    theta = f32(synth.mlp_init(5, last_scale=1.0))
    u = np.random.default_rng(seed).normal(0, 1, (f.n, 3))
    g = plan.position_vjp(_t(theta), pos, q, feat, vec, _t(u))
    ref = odip.position_vjp(theta, f32(f.pos), f32(f.q), f.box, 5.0, f32(u))
    e = rms_rel(host(g), ref)
    s = float(np.abs(host(g).sum(axis=0)).max() / np.sqrt(np.mean(ref ** 2)))
    print("vjp", n, f"{e:.2e}", "sum", f"{s:.2e}", flush=True)
    assert e <= RMS_REL_TOL
    assert s <= 1e-3 * np.sqrt(n)


def test_conservative_force_parity():
    """F = -(dU/dr + dip_position_vjp(dU/dmu)) with the GPU model against the
    oracle's total derivative."""
    from paper_2606_01598_amd.dip import DipPlan
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f = synth.molten_box(24, 33, L=13.0)
    pol = np.where(f.q > 0, 0.15, 3.5)
    mesh, p, alpha, rc = (16, 16, 16), 6, 0.35, 6.0
    pos, q, a = f32(f.pos), f32(f.q), f32(pol)
    theta = f32(synth.mlp_init(6, last_scale=1.0))
    F_ref, _, _ = odip.conservative_forces(theta, pos, q, a, f.box, mesh, p, alpha, rc, 5.0)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pme = Plan(mesh, p, alpha, max_atoms=f.n, keep_phi=True)
    polp = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    dip = DipPlan(f.box, f.n, cutoff=5.0)
    tp, tq, ta, th = _t(pos), _t(q), _t(a), _t(theta)
    feat, vec = dip.features(tp, tq)
    mu = dip.forward(th, feat, vec)
    s = polp.model(pme, tp, tq, mu, ta, box)
    F = -(s["dU_dpos"] + dip.position_vjp(th, tp, tq, feat, vec, s["dU_dmu"].contiguous()))
    e = rms_rel(host(F), F_ref)
    print("conservative force", f"{e:.2e}", flush=True)
    assert e <= RMS_REL_TOL
