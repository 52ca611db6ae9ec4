"""Autotuner of the plan geometry for the batched path.

For every distinct key (GPU architecture, mesh, order, atom-count bucket of
powers of two) it times candidates on a representative box with the library's
launch timer (the binning, spread, FFT and gather kernels of one forward +
Hessian-vector product step) and keeps the fastest.  The search is by
coordinates: first the spread/gather tile target (with the default FFT lines),
then the FFT lines per workgroup of the x pass (pme_desc_t.fft_lines) for the
best tile.  Results are cached in a JSON file so that later runs configure
plans without timing.
"""
from __future__ import annotations

import json
import math
import os
from typing import NamedTuple

import torch

from .pme import Plan

CANDIDATES = ((8, 8, 16), (8, 16, 16), (12, 12, 16), (16, 16, 16), (8, 8, 8), (16, 16, 8))
LINES = (4, 8, 16, 24, 32)
TIMED = ("bin", "bin_tangent", "spread", "spread_tangent", "fft_r2c", "fft_x", "fft_c2r",
         "gather", "gather_hvp")
VERSION = 2          # cache entries of other versions are timed again


class Config(NamedTuple):
    tile: tuple
    fft_lines: int   # 0: the library's default


def default_cache() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "pme_mi355x", "tiles.json")


def _key(arch, mesh, order, n) -> str:
    bucket = 1 << max(0, int(round(math.log2(max(1, n)))))
    return f"v{VERSION}|{arch}|{mesh[0]}x{mesh[1]}x{mesh[2]}|p{order}|n{bucket}"


def _time_candidate(cfg, mesh, order, alpha, pos, q, mu, box, v, steps):
    plan = Plan(mesh, order, alpha, max_atoms=max(1, pos.shape[0]), tile=cfg.tile,
                fft_lines=cfg.fft_lines or None)
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
         candidates=CANDIDATES, lines=LINES):
    """boxes: list of dicts (mesh, pos, q, mu, box, v) with device tensors, v the
    cotangents (v_pos, v_q, v_mu).  Returns (a Config per box, number of keys
    timed)."""
    path = cache_path or default_cache()
    cache = {}
    if os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    configs, timed = [], 0
    for b in boxes:
        key = _key(arch, b["mesh"], order, b["pos"].shape[0])
        if key not in cache:
            args = (b["mesh"], order, alpha, b["pos"], b["q"], b["mu"], b["box"], b["v"], steps)
            best = None
            for cand in candidates:
                cfg = Config(tuple(cand), 0)
                t = _time_candidate(cfg, *args)
                if best is None or t < best[0]:
                    best = (t, cfg)
            for k in lines:
                cfg = Config(best[1].tile, int(k))
                t = _time_candidate(cfg, *args)
                if t < best[0]:
                    best = (t, cfg)
            cache[key] = {"tile": list(best[1].tile), "fft_lines": best[1].fft_lines,
                          "ms": best[0]}
            timed += 1
        configs.append(Config(tuple(cache[key]["tile"]), int(cache[key]["fft_lines"])))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return configs, timed
