"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws numbers: positions, charges, dipoles, cells and the
batch layout of the molten-salt-like workloads.  It contains none of the
method's arithmetic (no spline weights, transforms, Green's function or
energies), so that the CPU oracle and the HIP path can both consume the same
arrays without sharing any computation.

Workloads (stand-ins for the paper's liquid-NaCl data of Sec. 3.2 and the
replicated supercells used for timing, which are not available):

* ``rocksalt``    -- NaCl conventional cells, optional Gaussian displacements.
* ``molten_box``  -- N ions (+1/-1, half each) placed uniformly at random with a
                     minimum periodic pair distance (random sequential
                     addition) at the density of molten NaCl, dipoles drawn
                     from N(0, sigma^2) per component.
* ``batch_boxes`` -- many molten boxes whose atom counts are log-uniform.

All generators use ``numpy.random.default_rng(seed)`` (PCG64) and return
float64 arrays; callers cast to float32 for the GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ions per cubic Angstrom of the molten-salt boxes: 1000 ions in a 31.5 A cube
MOLTEN_DENSITY = 1000.0 / 31.5 ** 3
ROCKSALT_A = 5.64


@dataclass
class Frame:
    pos: np.ndarray      # (N, 3) Angstrom, Cartesian
    q: np.ndarray        # (N,)  e
    mu: np.ndarray       # (N, 3) e*Angstrom
    box: np.ndarray      # (3, 3) rows are lattice vectors, Angstrom

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def rocksalt(ncell: int = 2, a: float = ROCKSALT_A, sigma: float = 0.1,
             seed: int = 0, displaced: bool = True) -> Frame:
    """ncell^3 conventional rock-salt cells: Na on fcc sites, Cl at +(a/2,0,0)."""
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    cells = np.array([[i, j, k] for i in range(ncell) for j in range(ncell)
                      for k in range(ncell)], dtype=float)
    na = (cells[:, None, :] + fcc[None, :, :]).reshape(-1, 3) * a
    cl = na + np.array([a / 2, 0.0, 0.0])
    pos = np.concatenate([na, cl])
    q = np.concatenate([np.ones(len(na)), -np.ones(len(cl))])
    L = ncell * a
    if displaced:
        rng = np.random.default_rng(seed)
        pos = pos + rng.normal(0.0, sigma, pos.shape)
    return Frame(pos=pos, q=q, mu=np.zeros_like(pos), box=np.eye(3) * L)


def molten_side(n: int) -> float:
    """Cube edge giving n ions at the molten-salt density."""
    return (n / MOLTEN_DENSITY) ** (1.0 / 3.0)


def _rsa(n: int, L: float, dmin: float, rng: np.random.Generator) -> np.ndarray:
    """Random sequential addition of n points in a periodic cube, min distance dmin.

    Candidates are drawn in batches; each is tested against the accepted points
    through a cell grid and against earlier candidates of its own batch.
    """
    ncell = max(1, int(L // dmin))
    h = L / ncell
    cap = max(4, int(math.ceil((h / dmin) ** 3 * 2.0)) + 2)
    grid = -np.ones((ncell, ncell, ncell, cap), dtype=np.int64)
    fill = np.zeros((ncell, ncell, ncell), dtype=np.int64)
    pts = np.empty((n, 3))
    count = 0
    d2 = dmin * dmin
    offs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    idle = 0
    if n * (math.pi / 6.0) * dmin ** 3 > 0.36 * L ** 3:
        raise ValueError("random sequential addition cannot reach this packing fraction")
    while count < n:
        idle += 1
        if idle > 2000:
            raise RuntimeError("random sequential addition jammed")
        need = n - count
        batch = int(min(max(64, need * 1.3 + 16), 1024))
        cand = rng.uniform(0.0, L, (batch, 3))
        cc = np.minimum((cand // h).astype(np.int64), ncell - 1)
        ok = np.ones(batch, dtype=bool)
        if count:
            nb = (cc[:, None, :] + offs[None, :, :]) % ncell           # (B,27,3)
            ids = grid[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(batch, -1)
            valid = ids >= 0
            other = pts[np.where(valid, ids, 0)]
            dv = cand[:, None, :] - other
            dv -= L * np.round(dv / L)
            close = (np.einsum('bkc,bkc->bk', dv, dv) < d2) & valid
            ok = ~close.any(axis=1)
        idx = np.nonzero(ok)[0]
        if idx.size > 1:
            c = cand[idx]
            dv = c[:, None, :] - c[None, :, :]
            dv -= L * np.round(dv / L)
            conflict = np.triu(np.einsum('ijc,ijc->ij', dv, dv) < d2, k=1)
            keep = np.ones(idx.size, dtype=bool)
            for i in np.nonzero(conflict.any(axis=1))[0]:
                if keep[i]:
                    keep[np.nonzero(conflict[i])[0]] = False
            idx = idx[keep]
        for i in idx[:need]:
            cx, cy, cz = cc[i]
            if fill[cx, cy, cz] >= cap:
                continue
            grid[cx, cy, cz, fill[cx, cy, cz]] = count
            fill[cx, cy, cz] += 1
            pts[count] = cand[i]
            count += 1
            idle = 0
    return pts


def molten_box(n: int, seed: int, L: float | None = None, dmin: float = 2.2,
               mu_sigma: float = 0.1) -> Frame:
    """n ions (n/2 of each sign) uniformly random with min periodic distance dmin."""
    if n % 2:
        raise ValueError("molten_box needs an even ion count")
    rng = np.random.default_rng(seed)
    L = molten_side(n) if L is None else float(L)
    pos = _rsa(n, L, dmin, rng)
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])[rng.permutation(n)]
    mu = rng.normal(0.0, mu_sigma, (n, 3))
    return Frame(pos=pos, q=q, mu=mu, box=np.eye(3) * L)


def _is_5smooth(m: int) -> bool:
    for f in (2, 3, 5):
        while m % f == 0:
            m //= f
    return m == 1


def nearest_smooth(x: float) -> int:
    """5-smooth integer nearest to x (ties go to the larger)."""
    lo = int(math.floor(x))
    best = None
    for m in range(max(1, lo - 64), lo + 65):
        if not _is_5smooth(m):
            continue
        if best is None or abs(m - x) < abs(best - x) or (abs(m - x) == abs(best - x) and m > best):
            best = m
    return best


def batch_boxes(n_boxes: int = 64, seed: int = 6, nmin: int = 64, nmax: int = 4096,
                mesh_lo: int = 16, mesh_hi: int = 64, mu_sigma: float = 0.1):
    """Boxes with log-uniform even atom counts at molten density; mesh ~1 A/point.

    Returns (frames, meshes) with meshes[b] = (M, M, M).
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(nmin), math.log(nmax), n_boxes)
    counts = [max(2, 2 * int(round(math.exp(v) / 2))) for v in u]
    seeds = rng.integers(0, 2 ** 31 - 1, n_boxes)
    frames, meshes = [], []
    for nb, sd in zip(counts, seeds):
        f = molten_box(nb, int(sd), mu_sigma=mu_sigma)
        frames.append(f)
        m = min(max(nearest_smooth(f.box[0, 0] / 1.0), mesh_lo), mesh_hi)
        meshes.append((m, m, m))
    return frames, meshes


def random_cotangents(n: int, seed: int, scale_r: float = 1.0, scale_q: float = 1.0,
                      scale_mu: float = 1.0):
    """Seeded cotangent vectors (v_r, v_q, v_mu) for Hessian-vector products."""
    rng = np.random.default_rng(seed)
    return (rng.normal(0, scale_r, (n, 3)), rng.normal(0, scale_q, n),
            rng.normal(0, scale_mu, (n, 3)))


def random_quadrupoles(n: int, seed: int, scale: float = 0.3, traceless: bool = False):
    """Seeded symmetric second moments Theta, stored as (n, 6) in the order xx, yy,
    zz, xy, xz, yz: Gaussian entries of standard deviation `scale` (e Angstrom^2)."""
    rng = np.random.default_rng(seed)
    th = rng.normal(0.0, scale, (n, 6))
    if traceless:
        th[:, :3] -= th[:, :3].mean(axis=1, keepdims=True)
    return th


def triclinic_cell(seed: int = 7, n: int = 8):
    """A small triclinic cell with random charges/dipoles (neutral)."""
    rng = np.random.default_rng(seed)
    box = np.array([[9.0, 0.0, 0.0], [2.1, 8.5, 0.0], [-1.3, 1.7, 10.2]])
    frac = rng.uniform(0, 1, (n, 3))
    pos = frac @ box
    q = rng.normal(0, 1, n)
    q -= q.mean()
    mu = rng.normal(0, 0.2, (n, 3))
    return Frame(pos=pos, q=q, mu=mu, box=box)


def mlp_init(seed: int, layers=((64, 34), (64, 64), (16, 64)), last_scale: float = 0.1):
    """Seeded initial parameters of a SiLU MLP, flat in the order W1 b1 W2 b2 W3 b3:
    Glorot-uniform weights (the last layer scaled by `last_scale`), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (fo, fi) in enumerate(layers):
        lim = math.sqrt(6.0 / (fi + fo)) * (last_scale if k == len(layers) - 1 else 1.0)
        parts.append(rng.uniform(-lim, lim, (fo, fi)).reshape(-1))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def charge_head_init(seed: int, hidden: int = 64, nfeat: int = 34, last_scale: float = 0.1,
                     bias_scale: float = 0.0):
    """Seeded initial parameters of the charge head, flat in the order W1 b1 w2:
    Glorot-uniform weights (the output layer scaled by `last_scale`) and biases
    uniform in +-bias_scale."""
    rng = np.random.default_rng(seed)
    lim1 = math.sqrt(6.0 / (nfeat + hidden))
    lim2 = math.sqrt(6.0 / (hidden + 1)) * last_scale
    return np.concatenate([rng.uniform(-lim1, lim1, hidden * nfeat),
                           rng.uniform(-bias_scale, bias_scale, hidden),
                           rng.uniform(-lim2, lim2, hidden)])
