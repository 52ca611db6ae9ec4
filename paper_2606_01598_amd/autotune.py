"""Tile autotuner for the spread and gather kernels.

For every distinct key (GPU architecture, mesh, order, atom-count bucket of
powers of two) it times candidate tile targets on a representative box with
the library's launch timer (the binning, spread and gather kernels of one
forward + Hessian-vector product step) and keeps the fastest.  Results are cached
in a JSON file so that later runs pick tiles without timing.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .pme import Plan

CANDIDATES = ((8, 8, 16), (8, 16, 16), (12, 12, 16), (16, 16, 16), (8, 8, 8), (16, 16, 8))
TIMED = ("bin", "bin_tangent", "spread", "spread_tangent", "gather", "gather_hvp")


def default_cache() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "pme_mi355x", "tiles.json")


def _key(arch, mesh, order, n) -> str:
    bucket = 1 << max(0, int(round(math.log2(max(1, n)))))
    return f"{arch}|{mesh[0]}x{mesh[1]}x{mesh[2]}|p{order}|n{bucket}"


def _time_candidate(tile, mesh, order, alpha, pos, q, mu, box, v, steps):
    plan = Plan(mesh, order, alpha, max_atoms=max(1, pos.shape[0]), tile=tile)
    for _ in range(2):
        plan.forward(pos, q, mu, box)
        plan.backward(pos, q, mu, box, *v)
    total = 0.0
    for kind in TIMED:
        plan.timer(kind)
        for _ in range(steps):
            plan.forward(pos, q, mu, box)
            plan.backward(pos, q, mu, box, *v)
        _, ms = plan.timer_read()
        total += ms
    plan.timer(None)
    plan.status()
    return total / steps


def tune(boxes, order: int, alpha: float, cache_path: str | None = None, steps: int = 3,
         candidates=CANDIDATES):
    """boxes: list of dicts (mesh, pos, q, mu, box, v) with device tensors, v the
    cotangents (v_pos, v_q, v_mu).  Returns (tiles per box, number of keys timed)."""
    path = cache_path or default_cache()
    cache = {}
    if os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    tiles, timed = [], 0
    for b in boxes:
        key = _key(arch, b["mesh"], order, b["pos"].shape[0])
        if key not in cache:
            best = None
            for cand in candidates:
                t = _time_candidate(cand, b["mesh"], order, alpha, b["pos"], b["q"], b["mu"],
                                    b["box"], b["v"], steps)
                if best is None or t < best[0]:
                    best = (t, list(cand))
            cache[key] = {"tile": best[1], "ms": best[0]}
            timed += 1
        tiles.append(tuple(cache[key]["tile"]))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return tiles, timed
