"""Throughput of the PME hot path on one MI355X.

One step = pme_forward (E^lr, dE/dr, dE/dq, dE/dmu) + pme_backward (Hessian-vector
product with generic cotangents v_r, v_q, v_mu), inputs resident in HBM, on the
32,000-ion molten-salt box (L = 100.006 A, mesh 100^3, p = 6, alpha = 0.30 1/A).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Work is fixed per GPU ("weak" scaling); only N = 1 runs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (n_ions, seed, mesh, order, alpha)
    "32k": (32000, 3, (100, 100, 100), 6, 0.30),
    "8k": (8000, 2, (64, 64, 64), 6, 0.30),
    "128k": (128000, 4, (160, 160, 160), 6, 0.30),
    "1m": (1000000, 5, (320, 320, 320), 6, 0.30),
}

HBM_PEAK_GBS = 8000.0


def _args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="32k", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-baseline", type=int, default=1,
                    help="0 skips the oracle timing on the host")
    ap.add_argument("--cpu-steps", type=int, default=3)
    return ap.parse_args(argv)


def main(argv=None):
    args = _args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2
    import numpy as np
    import torch

    import synth
    from paper_2606_01598_amd.pme import Plan

    n, seed, mesh, p, alpha = WORKLOADS[args.workload]
    frame = synth.molten_box(n, seed)
    dev = torch.device("cuda", 0)
    pos = torch.tensor(frame.pos, dtype=torch.float32, device=dev)
    q = torch.tensor(frame.q, dtype=torch.float32, device=dev)
    mu = torch.tensor(frame.mu, dtype=torch.float32, device=dev)
    box = torch.tensor(frame.box, dtype=torch.float64, device=dev)
    v = synth.random_cotangents(n, 11, scale_r=0.1)
    vr, vq, vm = (torch.tensor(x, dtype=torch.float32, device=dev) for x in v)
    plan = Plan(mesh, p, alpha, max_atoms=n, keep_phi=True)
    fo = {"energy": torch.empty(3, dtype=torch.float64, device=dev),
          "dE_dpos": torch.empty(n, 3, device=dev), "dE_dq": torch.empty(n, device=dev),
          "dE_dmu": torch.empty(n, 3, device=dev)}
    bo = {"g_pos": torch.empty(n, 3, device=dev), "g_q": torch.empty(n, device=dev),
          "g_mu": torch.empty(n, 3, device=dev)}

    def step():
        plan.forward(pos, q, mu, box, out=fo)
        plan.backward(pos, q, mu, box, vr, vq, vm, out=bo)

    for _ in range(args.warmup):
        step()
    plan.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.status()
    ms = (t1 - t0) * 1e3 / args.steps
    value = n * args.steps / (t1 - t0) / 1e6

    line = {
        "metric": "PME q+mu fwd+bwd Matom-steps/s @32k atoms",
        "value": value,
        "unit": "Matom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"molten-salt box, {n} ions (+-1 e, mu ~ N(0, 0.1^2) e*A), "
                               f"cubic L={frame.box[0, 0]:.3f} A, mesh {mesh[0]}x{mesh[1]}x{mesh[2]}, "
                               f"p={p}, alpha={alpha}, forward + Hessian-vector product",
                   "atoms": n, "mesh": list(mesh), "order": p, "alpha": alpha},
    }
    if args.cpu_baseline and args.workload == "32k":
        line["cpu_baseline"] = cpu_baseline(frame, mesh, p, alpha, v, args.cpu_steps)
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline(frame, mesh, p, alpha, v, steps):
    """The FP64 oracle (forward + HVP) timed on the host cores, on `steps` full steps."""
    import numpy as np

    from oracle import pme as opme
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    for _ in range(steps):
        opme.forward(frame.pos, frame.q, frame.mu, frame.box, mesh, p, alpha)
        opme.hvp(frame.pos, frame.q, frame.mu, frame.box, mesh, p, alpha, *v)
    dt = time.perf_counter() - t0
    return {"value": frame.n * steps / dt / 1e6, "unit": "Matom-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} full forward+HVP steps of the same {frame.n}-ion workload "
                      f"({dt:.1f} s)"}


if __name__ == "__main__":
    sys.exit(main())
