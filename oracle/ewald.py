"""Explicit Ewald summation for point charges and point dipoles (FP64).

The conventional baseline the paper validates its PME against (Sec. 2.3 and
the charged-dimer / molten-NaCl comparisons of Sec. 3): a real-space erfc pair
sum over periodic images, a direct sum over reciprocal vectors inside a cutoff
sphere, and the charge and dipole self terms (Eqs. self_q, self_mu).  Tin-foil
boundary conditions (no surface term).  The k-space part uses the screened
kernel of Eq. green; the structure factor of charges and dipoles is

    S(k) = sum_j (q_j + i mu_j . k) exp(i k . r_j),
    E_rec = (2 pi / V) sum_{k != 0, |k| < k_c} exp(-k^2 / 4 a^2) / k^2 |S(k)|^2.

Real-space pair energy for R = r_i - r_j + n C (Smith's B_l functions):

    U = q_i q_j B0 + (q_i mu_j - q_j mu_i) . R B1 + (mu_i . mu_j) B1
        - (mu_i . R)(mu_j . R) B2,
    B0 = erfc(a R)/R,
    B_l = [(2l-1) B_{l-1} + (2 a^2)^l exp(-a^2 R^2) / (a sqrt(pi))] / R^2,

and grad_R B_l = -R B_{l+1}.  Cutoffs are set from a tolerance eps:
erfc(a r_c) <= eps and k_c = 2 a sqrt(ln(1/eps)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erfc


@dataclass
class EwaldResult:
    e_real: float
    e_recip: float
    e_self_q: float
    e_self_mu: float
    e_background: float
    dE_dpos: np.ndarray
    dE_dq: np.ndarray
    dE_dmu: np.ndarray

    @property
    def energy(self) -> float:
        return self.e_real + self.e_recip + self.e_self_q + self.e_self_mu + self.e_background

    @property
    def long_range(self) -> float:
        """The part PME approximates: reciprocal sum plus self terms."""
        return self.e_recip + self.e_self_q + self.e_self_mu


def real_cutoff(alpha: float, eps: float) -> float:
    lo, hi = 0.0, 1.0
    while erfc(alpha * hi) > eps:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if erfc(alpha * mid) > eps:
            lo = mid
        else:
            hi = mid
    return hi


def _bl(r, alpha, lmax):
    """B_0 .. B_lmax at distances r (array)."""
    r2 = r * r
    g = np.exp(-alpha * alpha * r2) / (alpha * math.sqrt(math.pi))
    out = [erfc(alpha * r) / r]
    for l in range(1, lmax + 1):
        out.append(((2 * l - 1) * out[-1] + (2.0 * alpha * alpha) ** l * g) / r2)
    return out


def _real_space(pos, q, mu, C, alpha, rc, want_grad):
    n = pos.shape[0]
    recip_len = np.linalg.norm(np.linalg.inv(C), axis=0)    # |b_a| / 2pi
    nmax = [int(math.ceil(rc * recip_len[a])) for a in range(3)]
    shifts = np.array([[i, j, k] for i in range(-nmax[0], nmax[0] + 1)
                       for j in range(-nmax[1], nmax[1] + 1)
                       for k in range(-nmax[2], nmax[2] + 1)], dtype=np.float64) @ C
    e = 0.0
    gpos = np.zeros((n, 3))
    gq = np.zeros(n)
    gmu = np.zeros((n, 3))
    chunk = max(1, 2_000_000 // max(1, n * len(shifts)))
    for s in range(0, n, chunk):
        ii = np.arange(s, min(n, s + chunk))
        R = (pos[ii, None, None, :] - pos[None, :, None, :]) + shifts[None, None, :, :]
        r = np.sqrt(np.einsum('ijsc,ijsc->ijs', R, R))
        mask = r < rc
        self_img = (ii[:, None] == np.arange(n)[None, :])[:, :, None] & (r < 1e-12)
        mask &= ~self_img
        if not mask.any():
            continue
        ia, ja, sa = np.nonzero(mask)
        Rv = R[ia, ja, sa]
        rv = r[ia, ja, sa]
        B0, B1, B2, B3 = _bl(rv, alpha, 3)
        qi, qj = q[ii[ia]], q[ja]
        mi, mj = mu[ii[ia]], mu[ja]
        mir = np.einsum('pc,pc->p', mi, Rv)
        mjr = np.einsum('pc,pc->p', mj, Rv)
        mm = np.einsum('pc,pc->p', mi, mj)
        U = qi * qj * B0 + (qi * mjr - qj * mir) * B1 + mm * B1 - mir * mjr * B2
        e += 0.5 * float(np.sum(U))
        if not want_grad:
            continue
        gi = ii[ia]
        np.add.at(gq, gi, qj * B0 + mjr * B1)
        np.add.at(gmu, gi, (-qj * B1 - mjr * B2)[:, None] * Rv + B1[:, None] * mj)
        cross = qi * mjr - qj * mir
        gR = ((-qi * qj * B1 - cross * B2 - mm * B2 + mir * mjr * B3)[:, None] * Rv
              + B1[:, None] * (qi[:, None] * mj - qj[:, None] * mi)
              - B2[:, None] * (mi * mjr[:, None] + mj * mir[:, None]))
        notself = gi != ja
        np.add.at(gpos, gi[notself], gR[notself])
    return e, gpos, gq, gmu


def _kvectors(C, kc):
    Cinv = np.linalg.inv(C)
    recip = 2.0 * math.pi * Cinv.T
    hmax = [int(math.ceil(kc * np.linalg.norm(C[a]) / (2.0 * math.pi))) for a in range(3)]
    h = np.array([[i, j, k] for i in range(-hmax[0], hmax[0] + 1)
                  for j in range(-hmax[1], hmax[1] + 1)
                  for k in range(-hmax[2], hmax[2] + 1)
                  if (i, j, k) != (0, 0, 0)], dtype=np.float64)
    kv = h @ recip
    k2 = np.einsum('kc,kc->k', kv, kv)
    keep = k2 < kc * kc
    return kv[keep], k2[keep]


def _recip_space(pos, q, mu, C, alpha, kc, want_grad):
    n = pos.shape[0]
    V = abs(np.linalg.det(C))
    kv, k2 = _kvectors(C, kc)
    f = np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    e = 0.0
    gpos = np.zeros((n, 3))
    gq = np.zeros(n)
    gmu = np.zeros((n, 3))
    chunk = max(1, 4_000_000 // max(1, n))
    for s in range(0, len(kv), chunk):
        k = kv[s:s + chunk]
        fk = f[s:s + chunk]
        ph = np.exp(1j * (pos @ k.T))                     # (n, K)
        amp = q[:, None] + 1j * (mu @ k.T)                # q_j + i mu_j . k
        S = np.sum(amp * ph, axis=0)
        e += 2.0 * math.pi / V * float(np.sum(fk * np.abs(S) ** 2))
        if not want_grad:
            continue
        w = (4.0 * math.pi / V) * fk * np.conj(S)         # 2 * (2pi/V) f conj(S)
        base = ph * w[None, :]                            # (n, K)
        gq += np.real(base.sum(axis=1))
        gmu += np.real((1j * base) @ k)
        gpos += np.real((1j * amp * base) @ k)
    return e, gpos, gq, gmu


def ewald(pos, q, mu, box, alpha, eps=1e-14, rc=None, kc=None, background=False,
          want_grad=True, prefactor=1.0) -> EwaldResult:
    """Full Ewald energy and gradients of charges q and point dipoles mu."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    C = np.asarray(box, dtype=np.float64).reshape(3, 3)
    V = abs(np.linalg.det(C))
    rc = real_cutoff(alpha, eps) if rc is None else rc
    kc = 2.0 * alpha * math.sqrt(math.log(1.0 / eps)) if kc is None else kc
    er, gpr, gqr, gmr = _real_space(pos, q, mu, C, alpha, rc, want_grad)
    ek, gpk, gqk, gmk = _recip_space(pos, q, mu, C, alpha, kc, want_grad)
    sq = -alpha / math.sqrt(math.pi)
    smu = -2.0 * alpha ** 3 / (3.0 * math.sqrt(math.pi))
    eb = 0.0
    if background:
        eb = -math.pi * float(np.sum(q)) ** 2 / (2.0 * V * alpha * alpha)
    gq = gqr + gqk + 2.0 * sq * q
    if background:
        gq = gq - math.pi * float(np.sum(q)) / (V * alpha * alpha)
    gmu = gmr + gmk + 2.0 * smu * mu
    return EwaldResult(prefactor * er, prefactor * ek, prefactor * sq * float(np.sum(q * q)),
                       prefactor * smu * float(np.sum(mu * mu)), prefactor * eb,
                       prefactor * (gpr + gpk), prefactor * gq, prefactor * gmu)


def ewald_long_range(pos, q, mu, box, alpha, eps=1e-14, kc=None, prefactor=1.0):
    """Reciprocal sum + self terms only (the quantity PME approximates), with gradients."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    C = np.asarray(box, dtype=np.float64).reshape(3, 3)
    kc = 2.0 * alpha * math.sqrt(math.log(1.0 / eps)) if kc is None else kc
    ek, gpk, gqk, gmk = _recip_space(pos, q, mu, C, alpha, kc, True)
    sq = -alpha / math.sqrt(math.pi)
    smu = -2.0 * alpha ** 3 / (3.0 * math.sqrt(math.pi))
    e = ek + sq * float(np.sum(q * q)) + smu * float(np.sum(mu * mu))
    return (prefactor * e, prefactor * gpk, prefactor * (gqk + 2 * sq * q),
            prefactor * (gmk + 2 * smu * mu))
