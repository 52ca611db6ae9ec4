"""GPU parity of the learned dipole head (include/dip.h) against the FP64 oracle
(oracle/dip.py), through the C ABI, and a training run showing what the trained
network gains over the method without it (dipoles set to zero).

Bar: relative RMS error <= 1e-4 of features, dipoles, parameter gradients and
the training gradient through the PME model; relative error <= 1e-4 of the
loss (a sum of squared differences, so it loses the digits the differences
cancel).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import RMS_REL_TOL, dev, f32, host, rel, rms_rel
from oracle import dip as odip
from oracle import pol as opol

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev())


def test_features_parity():
    from paper_2606_01598_amd.dip import DipPlan
    f = synth.molten_box(300, 31)
    plan = DipPlan(f.box, f.n, cutoff=5.0)
    feat, vec = plan.features(_t(f.pos), _t(f.q))
    x, V = odip.features(f32(f.pos), f32(f.q), f.box, 5.0)
    e1, e2 = rms_rel(host(feat), x), rms_rel(host(vec), V)
    print("features", f"{e1:.2e}", f"{e2:.2e}", flush=True)
    assert e1 <= RMS_REL_TOL and e2 <= RMS_REL_TOL


def test_network_forward_and_backward_parity():
    from paper_2606_01598_amd.dip import DipPlan
    f = synth.molten_box(200, 32)
    plan = DipPlan(f.box, f.n, cutoff=5.0)
    x, V = odip.features(f32(f.pos), f32(f.q), f.box, 5.0)
    theta = f32(synth.mlp_init(5, last_scale=1.0))
    mu = plan.forward(_t(theta), _t(x), _t(V))
    mu_ref, _, cache = odip.dipoles(theta, f32(x), f32(V))
    e_mu = rms_rel(host(mu), mu_ref)
    rng = np.random.default_rng(4)
    gs = [rng.normal(0, 1, (f.n, 3)) for _ in range(3)]
    g = plan.backward(_t(theta), _t(x), _t(V), *[_t(a) for a in gs])
    gw = np.einsum('nd,ncd->nc', sum(f32(a) for a in gs), f32(V))
    g_ref = odip.mlp_backward(theta, cache, gw)
    e_g = rms_rel(host(g), g_ref)
    print("mlp", f"{e_mu:.2e}", f"{e_g:.2e}", flush=True)
    assert e_mu <= RMS_REL_TOL and e_g <= RMS_REL_TOL


def test_training_gradient_through_pme_parity():
    """Loss and parameter gradient of one training step (student dipoles -> PME
    model -> loss -> Hessian products -> network) against the oracle."""
    from paper_2606_01598_amd.dip import DipPlan, Trainer
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f = synth.molten_box(24, 33, L=13.0)
    pol = np.where(f.q > 0, 0.15, 3.5)
    mesh, p, alpha, rc = (16, 16, 16), 6, 0.35, 6.0
    pos, q, a = f32(f.pos), f32(f.q), f32(pol)
    mu_t = opol.induced_dipoles(pos, q, f.box, mesh, p, alpha, rc, a)
    U_t, dUdr_t, _ = opol.model(pos, q, mu_t, f.box, mesh, p, alpha, rc, a)
    x, V = odip.features(pos, q, f.box, 5.0)
    theta = f32(synth.mlp_init(6, last_scale=1.0))
    L_ref, g_ref, _ = odip.loss_and_grad(theta, f32(x), f32(V), pos, q, a, f.box, mesh, p, alpha,
                                         rc, {"U": U_t, "dUdr": dUdr_t, "mu": mu_t}, 1.0, 1.0, 0.5)
    box = torch.tensor(f.box, dtype=torch.float64, device=dev())
    pme = Plan(mesh, p, alpha, max_atoms=f.n, keep_phi=True)
    polp = PolPlan(f.box, alpha, rc, max_atoms=f.n)
    dip = DipPlan(f.box, f.n, cutoff=5.0)
    tr = Trainer(dip, polp, pme, box, theta, lr=0.0, lE=1.0, lF=1.0, lmu=0.5)
    b = {"pos": _t(pos), "q": _t(q), "pol": _t(a), "feat": _t(x), "vec": _t(V),
         "U": torch.tensor([U_t], dtype=torch.float64, device=dev()), "dUdr": _t(dUdr_t),
         "mu": _t(mu_t)}
    loss = float(host(tr.step(b))[0])
    e_L, e_g = rel(loss, L_ref), rms_rel(host(tr.g), g_ref)
    print("train-grad", f"{e_L:.2e}", f"{e_g:.2e}", flush=True)
    assert e_L <= 1e-4 and e_g <= RMS_REL_TOL


def test_training_beats_zero_dipoles():
    """A short training run on GPU teacher data (self-consistent Thole dipoles of
    small molten-salt boxes): the student's force error on held-out boxes falls
    below that of the same model with the dipoles left at zero."""
    from paper_2606_01598_amd.dip import DipPlan, Trainer
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    L = synth.molten_side(192)
    mesh, p, alpha, rc = (20, 20, 20), 6, 0.35, 6.0
    box_np = np.eye(3) * L
    box = torch.tensor(box_np, dtype=torch.float64, device=dev())
    n = 192
    pme = Plan(mesh, p, alpha, max_atoms=n, keep_phi=True)
    polp = PolPlan(box_np, alpha, rc, max_atoms=n)
    dip = DipPlan(box_np, n, cutoff=5.0)
    boxes = []
    for seed in range(3000, 3012):
        f = synth.molten_box(n, seed)
        pos, q = _t(f.pos), _t(f.q)
        a = _t(np.where(f.q > 0, 0.15, 3.5))
        mu, it, res = polp.scf(pme, pos, q, a, box, tol=1e-6, max_iter=300)
        t = polp.model(pme, pos, q, mu, a, box, dU_dmu=False)
        feat, vec = dip.features(pos, q)
        boxes.append({"pos": pos, "q": q, "pol": a, "feat": feat, "vec": vec, "U": t["energy"],
                      "dUdr": t["dU_dpos"], "mu": mu})
    train, val = boxes[:9], boxes[9:]

    def force_rmse(predict):
        errs = []
        for b in val:
            mu = predict(b)
            s = polp.model(pme, b["pos"], b["q"], mu, b["pol"], box, energy=False, dU_dmu=False)
            errs.append(float(torch.sqrt(torch.mean((s["dU_dpos"] - b["dUdr"]) ** 2))))
        return float(np.mean(errs))

    zero = force_rmse(lambda b: torch.zeros(n, 3, dtype=torch.float32, device=dev()))
    tr = Trainer(dip, polp, pme, box, synth.mlp_init(7), lr=3e-3, lE=1.0, lF=1.0)
    first = None
    for epoch in range(40):
        tot = 0.0
        for b in train:
            tot += float(host(tr.step(b))[0])
        first = tot if first is None else first
    student = force_rmse(lambda b: tr.predict(b["feat"], b["vec"]))
    print("force rmse: zero dipoles", f"{zero:.4e}", "student", f"{student:.4e}",
          "loss", f"{first:.3e}", "->", f"{tot:.3e}", flush=True)
    assert tot < first
    assert student < 0.8 * zero
