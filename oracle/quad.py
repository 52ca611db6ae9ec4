"""Quadrupole channel of the long-range energy (FP64 oracle; test infrastructure,
imported only by the tests, the smoke check and the benchmark's CPU baseline).

The paper names quadrupolar PME channels as the next extension of its Cartesian
multipoles (Sec. 4) without defining them.  The readings taken here:

* Each atom carries, besides q_i and mu_i, a symmetric Cartesian second moment
  Theta_i (six stored entries in the order xx, yy, zz, xy, xz, yz; it need not be
  traceless).  Its charge density is
      q_i delta - mu_i . grad delta + (1/2) Theta_i : grad grad delta   (at r_i),
  the limit of a cluster of point charges with sum q = q_i, sum q r = mu_i and
  sum q r r^T = Theta_i.
* Ewald structure factor: S(k) = sum_j (q_j + i mu_j . k - (1/2) k^T Theta_j k) e^{i k.r_j}.
* PME assignment (Sec. 2.3.2 extended by one order): the derivatives act on the
  atom's position, so the mesh density gains (1/2) sum_ab Q_ab d_a d_b W with
  Q = J Theta J^T in mesh coordinates, J[a][b] = N_a (C^-1)[b][a].
* Self terms (Eqs. self_q and self_mu extended): E_self removes the interaction of
  each multipole with its own screened field, -(1/2) O^+ O [erf(a u)/u] at u = 0
  with O^+ = q + mu . grad + (1/2) Theta : grad grad.  The series
  erf(a u)/u = (2/sqrt(pi)) (a - a^3 u^2 / 3 + a^5 u^4 / 10 - ...) gives
      E_self = - a/sqrt(pi) q^2 - 2a^3/(3 sqrt(pi)) |mu|^2
               + 2a^3/(3 sqrt(pi)) q tr(Theta)
               - a^5/(5 sqrt(pi)) [tr(Theta)^2 + 2 Theta:Theta].
* Gradients with respect to Theta are those of the six stored entries (an
  off-diagonal entry stands for both Theta_ab and Theta_ba).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import ewald as _ewald
from . import pme as _pme

# stored entries of Theta: (row, column)
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def theta_matrix(theta):
    """(n, 6) stored entries -> (n, 3, 3) symmetric matrices."""
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, 6)
    T = np.zeros((theta.shape[0], 3, 3))
    for k, (a, b) in enumerate(PAIRS):
        T[:, a, b] = theta[:, k]
        T[:, b, a] = theta[:, k]
    return T


def entries_gradient(G):
    """Gradient with respect to the six stored entries from the gradient G (n, 3, 3)
    with respect to independent matrix entries."""
    out = np.zeros((G.shape[0], 6))
    for k, (a, b) in enumerate(PAIRS):
        out[:, k] = G[:, a, b] if a == b else G[:, a, b] + G[:, b, a]
    return out


def _inputs(pos, q, mu, theta):
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    theta = np.zeros((n, 6)) if theta is None else np.asarray(theta, dtype=np.float64)
    return pos, q, mu, theta.reshape(n, 6)


# ----------------------------------------------------------------------------
# self terms
# ----------------------------------------------------------------------------

def self_energy(q, mu, theta, alpha):
    """(E_self_q, E_self_mu, E_self_theta); the last holds the q-Theta cross term."""
    sp = math.sqrt(math.pi)
    T = theta_matrix(theta)
    tr = np.trace(T, axis1=1, axis2=2)
    e_q = -alpha / sp * float(np.sum(q * q))
    e_mu = -2.0 * alpha ** 3 / (3.0 * sp) * float(np.sum(mu * mu))
    e_th = (2.0 * alpha ** 3 / (3.0 * sp) * float(np.sum(q * tr))
            - alpha ** 5 / (5.0 * sp) * float(np.sum(tr * tr + 2.0 * np.sum(T * T, axis=(1, 2)))))
    return e_q, e_mu, e_th


def self_gradients(q, mu, theta, alpha):
    """Gradients of the self terms with respect to q, mu and the stored Theta entries."""
    sp = math.sqrt(math.pi)
    c1 = 2.0 * alpha ** 3 / (3.0 * sp)
    c2 = alpha ** 5 / (5.0 * sp)
    T = theta_matrix(theta)
    tr = np.trace(T, axis1=1, axis2=2)
    gq = -2.0 * alpha / sp * q + c1 * tr
    gmu = -2.0 * c1 * mu
    # d/dT_ab (independent entries) of c1 q tr - c2 (tr^2 + 2 T:T)
    G = (c1 * q - 2.0 * c2 * tr)[:, None, None] * np.eye(3)[None] - 4.0 * c2 * T
    return gq, gmu, entries_gradient(G)


# ----------------------------------------------------------------------------
# PME with the quadrupole channel
# ----------------------------------------------------------------------------

def density(pos, q, mu, theta, box, mesh, p):
    """rho(n) = sum_i sum_stencil [q W + (J mu) . grad_x W + (1/2) (J Theta J^T) : grad_x grad_x W]."""
    pos, q, mu, theta = _inputs(pos, q, mu, theta)
    J = _pme.jacobian(box, mesh)
    d = mu @ J.T
    Q = np.einsum('ac,ncd,bd->nab', J, theta_matrix(theta), J)
    coeffs = {(0, 0, 0): q, (1, 0, 0): d[:, 0], (0, 1, 0): d[:, 1], (0, 0, 1): d[:, 2]}
    for a, b in PAIRS:
        key = [0, 0, 0]
        key[a] += 1
        key[b] += 1
        # (1/2) sum over both orders of an off-diagonal pair: Q_ab; diagonal: Q_aa / 2
        coeffs[tuple(key)] = Q[:, a, b] if a != b else 0.5 * Q[:, a, a]
    return _pme._spread_terms(pos, box, mesh, p, coeffs)


@dataclass
class QuadResult:
    e_recip: float
    e_self_q: float
    e_self_mu: float
    e_self_theta: float
    dE_dpos: np.ndarray
    dE_dq: np.ndarray
    dE_dmu: np.ndarray
    dE_dtheta: np.ndarray
    rho: np.ndarray
    phi: np.ndarray

    @property
    def energy(self) -> float:
        return self.e_recip + self.e_self_q + self.e_self_mu + self.e_self_theta


def forward(pos, q, mu, theta, box, mesh, p, alpha, gamma=1.0, prefactor=1.0) -> QuadResult:
    """E^lr of charges, dipoles and quadrupoles and its gradients.

    With S_k the order-k stencil sums of phi (x-space derivatives of W), d = J mu and
    Q = J Theta J^T:
      dE/dq     = S_0 / V + self
      dE/dmu    = J^T S_1 / V + self
      dE/dTheta = (1/2) J^T S_2 J / V + self      (independent entries; then stored)
      dE/dr     = J^T [q S_1 + S_2 d + (1/2) S_3 : Q] / V
    """
    pos, q, mu, theta = _inputs(pos, q, mu, theta)
    mesh = tuple(int(m) for m in mesh)
    _, _, V, _ = _pme.cell(box)
    J = _pme.jacobian(box, mesh)
    rho = density(pos, q, mu, theta, box, mesh, p)
    phi = _pme.potential(rho, _pme.influence(box, mesh, p, alpha, gamma))
    e_recip = float(np.sum(rho * phi)) / (2.0 * V)
    orders = _pme._orders(0) + _pme._orders(1) + _pme._orders(2) + _pme._orders(3)
    S = _pme._stencil_sums(pos, box, mesh, p, phi, orders)
    g1 = _pme._grad_vec(S)
    H = _pme._hess_mat(S)
    d = mu @ J.T
    Q = np.einsum('ac,ncd,bd->nab', J, theta_matrix(theta), J)
    t3 = np.zeros_like(d)                       # (1/2) sum_ab Q_ab S_abc
    for a in range(3):
        for b in range(3):
            for c in range(3):
                key = [0, 0, 0]
                key[a] += 1
                key[b] += 1
                key[c] += 1
                t3[:, c] += 0.5 * Q[:, a, b] * S[tuple(key)]
    sq, smu, sth = self_gradients(q, mu, theta, alpha)
    e_q, e_mu, e_th = self_energy(q, mu, theta, alpha)
    dE_dq = S[(0, 0, 0)] / V + sq
    dE_dmu = (g1 @ J) / V + smu
    G = 0.5 * np.einsum('ac,nab,bd->ncd', J, H, J) / V
    dE_dtheta = entries_gradient(G) + sth
    dE_dpos = (q[:, None] * g1 + np.einsum('nab,nb->na', H, d) + t3) @ J / V
    pf = prefactor
    return QuadResult(pf * e_recip, pf * e_q, pf * e_mu, pf * e_th, pf * dE_dpos, pf * dE_dq,
                      pf * dE_dmu, pf * dE_dtheta, rho, phi)


def energy(pos, q, mu, theta, box, mesh, p, alpha, gamma=1.0, prefactor=1.0) -> float:
    pos, q, mu, theta = _inputs(pos, q, mu, theta)
    _, _, V, _ = _pme.cell(box)
    rho = density(pos, q, mu, theta, box, mesh, p)
    phi = _pme.potential(rho, _pme.influence(box, mesh, p, alpha, gamma))
    return prefactor * (float(np.sum(rho * phi)) / (2.0 * V) + sum(self_energy(q, mu, theta, alpha)))


# ----------------------------------------------------------------------------
# explicit Ewald reciprocal sum with the quadrupole channel
# ----------------------------------------------------------------------------

@dataclass
class EwaldQuad:
    e_recip: float
    e_self: float
    dE_dpos: np.ndarray
    dE_dq: np.ndarray
    dE_dmu: np.ndarray
    dE_dtheta: np.ndarray

    @property
    def energy(self) -> float:
        return self.e_recip + self.e_self


def ewald_long_range(pos, q, mu, theta, box, alpha, eps=1e-14, kc=None, prefactor=1.0):
    """Reciprocal sum over |k| < k_c plus self terms, with gradients:
    E_rec = (2 pi / V) sum_k exp(-k^2/4a^2)/k^2 |S(k)|^2."""
    pos, q, mu, theta = _inputs(pos, q, mu, theta)
    n = pos.shape[0]
    C = np.asarray(box, dtype=np.float64).reshape(3, 3)
    V = abs(np.linalg.det(C))
    kc = 2.0 * alpha * math.sqrt(math.log(1.0 / eps)) if kc is None else kc
    kv, k2 = _ewald._kvectors(C, kc)
    f = np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    T = theta_matrix(theta)
    e = 0.0
    gpos = np.zeros((n, 3))
    gq = np.zeros(n)
    gmu = np.zeros((n, 3))
    gT = np.zeros((n, 3, 3))
    chunk = max(1, 2_000_000 // max(1, n))
    for s in range(0, len(kv), chunk):
        k = kv[s:s + chunk]
        fk = f[s:s + chunk]
        ph = np.exp(1j * (pos @ k.T))                               # (n, K)
        kTk = np.einsum('ka,nab,kb->nk', k, T, k)
        amp = q[:, None] + 1j * (mu @ k.T) - 0.5 * kTk
        S = np.sum(amp * ph, axis=0)
        e += 2.0 * math.pi / V * float(np.sum(fk * np.abs(S) ** 2))
        w = (4.0 * math.pi / V) * fk * np.conj(S)
        base = ph * w[None, :]
        gq += np.real(base.sum(axis=1))
        gmu += np.real((1j * base) @ k)
        gpos += np.real((1j * amp * base) @ k)
        gT += -0.5 * np.real(np.einsum('nk,ka,kb->nab', base, k, k))
    e_q, e_mu, e_th = self_energy(q, mu, theta, alpha)
    sq, smu, sth = self_gradients(q, mu, theta, alpha)
    pf = prefactor
    return EwaldQuad(pf * e, pf * (e_q + e_mu + e_th), pf * gpos, pf * (gq + sq), pf * (gmu + smu),
                     pf * (entries_gradient(gT) + sth))
