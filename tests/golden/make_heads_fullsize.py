"""Write the oracle's values for one training step of both learned heads on
conservative forces at the size of the learned-head workload: a 4096-ion
molten-salt box (synth.molten_box(4096, 2000), the first held-out box of the
training run), polarizabilities 0.15 / 3.5 A^3, mesh 50^3, p = 6, alpha = 0.30,
real-space cutoff 10 A, feature cutoff 5 A (Secs. 2.2 and 2.4: Eqs. charge_pred,
dipole_pred, forces, loss).

    python tests/golden/make_heads_fullsize.py

The parameters are synth.mlp_init(7, last_scale=1.0) and
synth.charge_head_init(8, last_scale=1.0, bias_scale=0.5); positions are rounded
to float32 as the GPU sees them.  The loss compares the student with a fixed
target (energy 0, forces 0, dipoles 0; lE = lF = 1, lmu = 0.5), which is enough to
exercise every term of the gradient.  The file keeps the loss, both parameter
gradients (the dipole head's at a seeded sample of entries), and the charges,
dipoles and conservative forces of a seeded sample of atoms.  A second case is
the dipole head alone on Hellmann-Feynman forces (oracle/dip.py loss_and_grad,
the training step of the learned dipole head): its loss and the same sample of
its parameter gradient, lines prefixed hf_.  Only oracle/ and synth/ are called
(about 6 minutes on 8 cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dip as odip  # noqa: E402
from oracle import heads as oh  # noqa: E402

N, SEED = 4096, 2000
MESH, P, ALPHA, RC, RC_FEAT = (50, 50, 50), 6, 0.30, 10.0, 5.0
THETA_SEED, THQ_SEED = 7, 8
LOSS = dict(lE=1.0, lF=1.0, lmu=0.5)
SAMPLE_ATOMS, SAMPLE_PARAMS, SAMPLE_SEED = 256, 1024, 91
PATH = os.path.join(HERE, "heads_4096.txt")


def inputs():
    f = synth.molten_box(N, SEED)
    pos = np.asarray(f.pos, dtype=np.float32).astype(np.float64)
    z = np.asarray(f.q, dtype=np.float32).astype(np.float64)
    pol = np.where(z > 0, 0.15, 3.5)
    theta = np.asarray(synth.mlp_init(THETA_SEED, last_scale=1.0), np.float32).astype(np.float64)
    thq = np.asarray(synth.charge_head_init(THQ_SEED, last_scale=1.0, bias_scale=0.5),
                     np.float32).astype(np.float64)
    return f, pos, z, pol, theta, thq


def samples():
    rng = np.random.default_rng(SAMPLE_SEED)
    atoms = np.sort(rng.choice(N, SAMPLE_ATOMS, replace=False))
    params = np.sort(rng.choice(odip.NPARAM, SAMPLE_PARAMS, replace=False))
    return atoms, params


def teacher():
    return {"U": 0.0, "dUdr": np.zeros((N, 3)), "mu": np.zeros((N, 3))}


def main():
    t0 = time.time()
    f, pos, z, pol, theta, thq = inputs()
    L, g, gq = oh.loss_and_grad(theta, thq, pos, z, pol, f.box, MESH, P, ALPHA, RC, teacher(),
                                conservative=True, rc_feat=RC_FEAT, **LOSS)
    s = oh.student(theta, thq, pos, z, pol, f.box, MESH, P, ALPHA, RC, RC_FEAT)
    x, V = odip.features(pos, z, f.box, RC_FEAT)
    tch = teacher()
    L_hf, g_hf, _ = odip.loss_and_grad(theta, x, V, pos, z, pol, f.box, MESH, P, ALPHA, RC, tch,
                                       LOSS["lE"], LOSS["lF"], LOSS["lmu"])
    atoms, params = samples()
    with open(PATH, "w") as fh:
        fh.write(f"# FP64 oracle (oracle/heads.py loss_and_grad, student) on synth.molten_box({N}, "
                 f"{SEED}), box {float(f.box[0, 0])!r} A cubic, mesh 50^3, p=6, alpha=0.3, r_c=10, "
                 f"feature r_c=5;\n# parameters synth.mlp_init({THETA_SEED}, last_scale=1.0), "
                 f"synth.charge_head_init({THQ_SEED}, last_scale=1.0, bias_scale=0.5); "
                 f"target 0, lE=1, lF=1, lmu=0.5; conservative forces, both heads.\n")
        fh.write(f"# written by tests/golden/make_heads_fullsize.py ({time.time() - t0:.0f} s)\n")
        fh.write(f"loss {float(L)!r}\n")
        for k, v in zip(params, g[params]):
            fh.write(f"g_theta {int(k)} {float(v)!r}\n")
        for k, v in enumerate(gq):
            fh.write(f"g_thq {k} {float(v)!r}\n")
        fh.write(f"hf_loss {float(L_hf)!r}\n")
        for k, v in zip(params, g_hf[params]):
            fh.write(f"hf_g_theta {int(k)} {float(v)!r}\n")
        for i in atoms:
            F, m = s["F"][i], s["mu"][i]
            fh.write(f"atom {int(i)} {float(s['q'][i])!r} {float(m[0])!r} {float(m[1])!r} "
                     f"{float(m[2])!r} {float(F[0])!r} {float(F[1])!r} {float(F[2])!r}\n")
    print("wrote", PATH, f"{time.time() - t0:.0f} s")


def read_hf():
    """(loss, {index: dL/dtheta}) of the Hellmann-Feynman dipole-head case"""
    L, gt = None, {}
    with open(PATH) as fh:
        for ln in fh:
            w = ln.split()
            if w and w[0] == "hf_loss":
                L = float(w[1])
            elif w and w[0] == "hf_g_theta":
                gt[int(w[1])] = float(w[2])
    return L, gt


def read():
    """(loss, {index: dL/dtheta}, dL/dthq array, atoms, q, mu, F)"""
    L, gt, gq, at, q, mu, F = None, {}, {}, [], [], [], []
    with open(PATH) as fh:
        for ln in fh:
            if ln.startswith("#") or not ln.strip():
                continue
            w = ln.split()
            if w[0] == "loss":
                L = float(w[1])
            elif w[0] == "g_theta":
                gt[int(w[1])] = float(w[2])
            elif w[0] == "g_thq":
                gq[int(w[1])] = float(w[2])
            elif w[0] == "atom":
                at.append(int(w[1]))
                q.append(float(w[2]))
                mu.append([float(x) for x in w[3:6]])
                F.append([float(x) for x in w[6:9]])
    return (L, gt, np.array([gq[k] for k in range(len(gq))]), np.array(at), np.array(q),
            np.array(mu), np.array(F))


if __name__ == "__main__":
    main()
