"""Write the oracle's values for the full-size molten-salt workloads of the size
sweep (128,000 ions on a 160^3 mesh and 1,000,000 ions on a 320^3 mesh, p = 6,
alpha = 0.30; the supercell scaling of Sec. 3.2 with synthetic stand-ins for its
data), for the GPU parity tests that run at those sizes.

    python tests/golden/make_fullsize.py [128k] [1m]

For each workload the inputs are the seeded arrays the GPU receives (positions,
charges and dipoles from synth.molten_box, cotangents from
synth.random_cotangents), rounded to float32 as the GPU sees them.  The FP64
oracle (oracle/pme.py: forward for E^lr and its gradients, hvp for the
Hessian-vector product) runs on every atom; the file keeps the three energy
terms and the outputs of a seeded sample of atoms, which the GPU tests compare
one by one.  Only oracle/ and synth/ are called.
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
from oracle import pme as opme  # noqa: E402

# name: (ions, seed, mesh, order, alpha); cotangent seed 11 with scale_r 0.1
WORKLOADS = {
    "128k": (128000, 4, (160, 160, 160), 6, 0.30),
    "1m": (1000000, 5, (320, 320, 320), 6, 0.30),
}
COT_SEED = 11
SAMPLE = 256
SAMPLE_SEED = 77
COLUMNS = ("atom dE_dpos_x dE_dpos_y dE_dpos_z dE_dq dE_dmu_x dE_dmu_y dE_dmu_z "
           "g_pos_x g_pos_y g_pos_z g_q g_mu_x g_mu_y g_mu_z")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def path(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.txt")


def sample_indices(n: int) -> np.ndarray:
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, SAMPLE, replace=False))


def write(name: str) -> None:
    n, seed, mesh, p, alpha = WORKLOADS[name]
    t0 = time.time()
    f = synth.molten_box(n, seed)
    v = synth.random_cotangents(n, COT_SEED, scale_r=0.1)
    pos, q, mu = f32(f.pos), f32(f.q), f32(f.mu)
    t1 = time.time()
    ref = opme.forward(pos, q, mu, f.box, mesh, p, alpha)
    t2 = time.time()
    hv = opme.hvp(pos, q, mu, f.box, mesh, p, alpha, v_pos=f32(v[0]), v_q=f32(v[1]),
                  v_mu=f32(v[2]))
    t3 = time.time()
    idx = sample_indices(n)
    with open(path(name), "w") as fh:
        fh.write(f"# FP64 oracle (oracle/pme.py forward, hvp) on the molten-salt box of {n} ions,\n")
        fh.write(f"# synth.molten_box({n}, {seed}), box {float(f.box[0, 0])!r} A cubic, mesh "
                 f"{mesh[0]}x{mesh[1]}x{mesh[2]}, p={p}, alpha={alpha}, gamma=1;\n")
        fh.write(f"# cotangents synth.random_cotangents({n}, {COT_SEED}, scale_r=0.1); inputs "
                 "rounded to float32.\n")
        fh.write("# written by tests/golden/make_fullsize.py "
                 f"(inputs {t1 - t0:.0f} s, forward {t2 - t1:.0f} s, hvp {t3 - t2:.0f} s)\n")
        fh.write(f"energy {float(ref.e_recip)!r} {float(ref.e_self_q)!r} {float(ref.e_self_mu)!r}\n")
        fh.write(f"sample {SAMPLE} seed {SAMPLE_SEED}\n")
        fh.write(f"# {COLUMNS}\n")
        for i in idx:
            vals = ([ref.dE_dpos[i, k] for k in range(3)] + [ref.dE_dq[i]]
                    + [ref.dE_dmu[i, k] for k in range(3)] + [hv[0][i, k] for k in range(3)]
                    + [hv[1][i]] + [hv[2][i, k] for k in range(3)])
            fh.write(f"{int(i)} " + " ".join(repr(float(x)) for x in vals) + "\n")
    print(f"{name}: wrote {path(name)} ({t3 - t0:.0f} s)", flush=True)


def read(name: str):
    """(energy terms (3,), sampled atom indices (S,), outputs (S, 14) in COLUMNS order)."""
    energy, rows = None, []
    with open(path(name)) as fh:
        for line in fh:
            if line.startswith("#") or line.startswith("sample"):
                continue
            if line.startswith("energy"):
                energy = np.array([float(x) for x in line.split()[1:]])
                continue
            rows.append([float(x) for x in line.split()])
    a = np.array(rows)
    return energy, a[:, 0].astype(np.int64), a[:, 1:]


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        write(name)
