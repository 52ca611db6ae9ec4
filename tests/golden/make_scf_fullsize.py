"""Write the oracle's self-consistent teacher on the 4096-ion teacher box:
synth.molten_box(4096, 1000) (L = 50.4 A), polarizabilities 0.15 / 3.5 A^3, mesh
50^3, p = 6, alpha = 0.30, real-space cutoff 10 A (the polarizable model of the
teacher, Secs. 2.3-2.4, solved self-consistently).

    python tests/golden/make_scf_fullsize.py

The dipoles come from oracle/pol.py induced_dipoles_cg (plain CG with matrix-free
PME Hessian products, to |b - A mu| <= 1e-12 |b|; pinned to the dense solve on
small boxes), and the energy and forces from oracle/pol.py model at those dipoles.
Positions, charges and polarizabilities are rounded to float32 as the GPU sees
them.  The file keeps the energy U, the RMS dipole, the stationarity |dU/dmu| /
|field| of the forward calls, and the dipoles and forces of a seeded sample of
atoms.  Only oracle/ and synth/ are called (about a minute on 8 cores).
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
from oracle import pol as opol  # noqa: E402

N, SEED = 4096, 1000
MESH, P, ALPHA, RC = (50, 50, 50), 6, 0.30, 10.0
SAMPLE_ATOMS, SAMPLE_SEED = 256, 92
PATH = os.path.join(HERE, "scf_4096.txt")


def inputs():
    f = synth.molten_box(N, SEED)
    pos = np.asarray(f.pos, dtype=np.float32).astype(np.float64)
    q = np.asarray(f.q, dtype=np.float32).astype(np.float64)
    pol = np.asarray(np.where(f.q > 0, 0.15, 3.5), np.float32).astype(np.float64)
    return f, pos, q, pol


def samples():
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(N, SAMPLE_ATOMS, replace=False))


def main():
    t0 = time.time()
    f, pos, q, pol = inputs()
    mu, it = opol.induced_dipoles_cg(pos, q, f.box, MESH, P, ALPHA, RC, pol, tol=1e-12)
    U, dUdr, dUdmu = opol.model(pos, q, mu, f.box, MESH, P, ALPHA, RC, pol)
    field = dUdmu - mu / pol[:, None]
    stat = float(np.linalg.norm(dUdmu) / np.linalg.norm(field))
    atoms = samples()
    with open(PATH, "w") as fh:
        fh.write(f"# FP64 oracle (oracle/pol.py induced_dipoles_cg, model) on synth.molten_box({N}, "
                 f"{SEED}), box {float(f.box[0, 0])!r} A cubic, mesh 50^3, p=6, alpha=0.3, "
                 f"r_c=10, polarizabilities 0.15 / 3.5 A^3;\n# CG to 1e-12 relative residual in "
                 f"{it} iterations; |dU/dmu| / |field| = {stat:.3e}.\n")
        fh.write(f"# written by tests/golden/make_scf_fullsize.py ({time.time() - t0:.0f} s)\n")
        fh.write(f"energy {float(U)!r}\n")
        fh.write(f"mu_rms {float(np.sqrt(np.mean(np.sum(mu * mu, axis=1))))!r}\n")
        for i in atoms:
            m, F = mu[i], -dUdr[i]
            fh.write(f"atom {int(i)} {float(m[0])!r} {float(m[1])!r} {float(m[2])!r} "
                     f"{float(F[0])!r} {float(F[1])!r} {float(F[2])!r}\n")
    print("wrote", PATH, it, f"{stat:.2e}", f"{time.time() - t0:.0f} s")


def read():
    """(energy, mu_rms, atoms, mu (k, 3), F (k, 3))"""
    E, m_rms, at, mu, F = None, None, [], [], []
    with open(PATH) as fh:
        for ln in fh:
            w = ln.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "energy":
                E = float(w[1])
            elif w[0] == "mu_rms":
                m_rms = float(w[1])
            elif w[0] == "atom":
                at.append(int(w[1]))
                mu.append([float(x) for x in w[2:5]])
                F.append([float(x) for x in w[5:8]])
    return E, m_rms, np.array(at), np.array(mu), np.array(F)


if __name__ == "__main__":
    main()
