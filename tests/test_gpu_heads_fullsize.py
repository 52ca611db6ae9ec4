"""Oracle parity of one training step of both learned heads on conservative
forces at the size of the learned-head workload (a 4096-ion box, mesh 50^3,
real-space cutoff 10 A; Eqs. charge_pred, dipole_pred, forces, loss): the GPU
Trainer (charge head, conservative forces) against the values
tests/golden/make_heads_fullsize.py wrote with the FP64 oracle on the same
seeded inputs: the loss, the charge head's whole parameter gradient and a seeded
sample of the dipole head's, and the charges, dipoles and conservative forces of
a seeded sample of atoms.

A second test does the same for the dipole head alone on Hellmann-Feynman forces
(the learned dipole head's training step) against oracle/dip.py.

Bar: 1e-4 relative for the loss and relative RMS for each compared array.
"""
import os
import sys

import numpy as np
import pytest
import torch

from gpu_util import RMS_REL_TOL, dev, host, rel, rms_rel

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_heads_fullsize as mh  # noqa: E402


def test_conservative_training_step_4096_ions():
    from paper_2606_01598_amd.dip import DipPlan, Trainer
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f, pos, z, pol, theta, thq = mh.inputs()
    print(f"case: conservative training step, {mh.N} ions, both heads", flush=True)
    d = dev()
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=d)
    box = torch.tensor(f.box, dtype=torch.float64, device=d)
    pme = Plan(mh.MESH, mh.P, mh.ALPHA, max_atoms=mh.N, keep_phi=True)
    polp = PolPlan(f.box, mh.ALPHA, mh.RC, max_atoms=mh.N)
    dip = DipPlan(f.box, mh.N, cutoff=mh.RC_FEAT)
    tp, tz = t(pos), t(z)
    feat, vec = dip.features(tp, tz)
    tr = Trainer(dip, polp, pme, box, theta, lr=0.0, qtheta0=thq, conservative=True, **mh.LOSS)
    zero = torch.zeros(mh.N, 3, dtype=torch.float32, device=d)
    b = {"pos": tp, "q": tz, "pol": t(pol), "feat": feat, "vec": vec,
         "U": torch.zeros(1, dtype=torch.float64, device=d), "dUdr": zero, "mu": zero}
    loss = float(host(tr.step(b))[0])
    L, gt, gq, atoms, q_ref, mu_ref, F_ref = mh.read()
    idx = np.array(sorted(gt))
    g_ref = np.array([gt[k] for k in idx])
    e_L = rel(loss, L)
    e_g = rms_rel(host(tr.g)[idx], g_ref)
    e_q = rms_rel(host(tr.gq), gq)
    ev = tr.evaluate(b)
    ii = torch.tensor(atoms, device=d)
    e_charge = rms_rel(host(ev["q"][ii]) - z[atoms], q_ref - z[atoms], floor=1e-3)
    e_mu = rms_rel(host(ev["mu"][ii]), mu_ref)
    e_F = rms_rel(-host(ev["dU_dpos"][ii]), F_ref)
    print("4096 ions", f"loss {e_L:.2e} g_theta {e_g:.2e} g_thq {e_q:.2e} q {e_charge:.2e} "
          f"mu {e_mu:.2e} F {e_F:.2e}", flush=True)
    assert e_L <= 1e-4
    assert max(e_g, e_q, e_charge, e_mu, e_F) <= RMS_REL_TOL


def test_hellmann_feynman_training_step_4096_ions():
    """The dipole head alone on Hellmann-Feynman forces (the training step of the
    learned dipole head: dip_backward with the PME and real-space mixed Hessian
    products) against oracle/dip.py at the same size."""
    from paper_2606_01598_amd.dip import DipPlan, Trainer
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan
    f, pos, z, pol, theta, _ = mh.inputs()
    print(f"case: Hellmann-Feynman training step, {mh.N} ions, dipole head", flush=True)
    d = dev()
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=d)
    box = torch.tensor(f.box, dtype=torch.float64, device=d)
    pme = Plan(mh.MESH, mh.P, mh.ALPHA, max_atoms=mh.N, keep_phi=True)
    polp = PolPlan(f.box, mh.ALPHA, mh.RC, max_atoms=mh.N)
    dip = DipPlan(f.box, mh.N, cutoff=mh.RC_FEAT)
    tp, tz = t(pos), t(z)
    feat, vec = dip.features(tp, tz)
    tr = Trainer(dip, polp, pme, box, theta, lr=0.0, **mh.LOSS)
    zero = torch.zeros(mh.N, 3, dtype=torch.float32, device=d)
    b = {"pos": tp, "q": tz, "pol": t(pol), "feat": feat, "vec": vec,
         "U": torch.zeros(1, dtype=torch.float64, device=d), "dUdr": zero, "mu": zero}
    loss = float(host(tr.step(b))[0])
    L, gt = mh.read_hf()
    idx = np.array(sorted(gt))
    e_L = rel(loss, L)
    e_g = rms_rel(host(tr.g)[idx], np.array([gt[k] for k in idx]))
    print("4096 ions HF", f"loss {e_L:.2e} g_theta {e_g:.2e}", flush=True)
    assert e_L <= 1e-4 and e_g <= RMS_REL_TOL
