"""Thole-damped polarizable point-charge model solved with PME (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The model is the teacher of the learned dipole head.
- The paper's own polarization is not self-consistent (Sec. 4). Here the induced dipoles are solved self-consistently.
- Thole damping is only cited in the paper's introduction. Its form follows the reading stated in the design notes: exponential damping with A = 0.39.

Model. With atomic polarizabilities a_i:

    U(mu) = E_lr(q, mu) + E_real(q, mu) + sum_i |mu_i|^2 / (2 a_i)

E_lr is the PME long-range energy of Secs. 2.3.1-2.3.5: E_recip plus the self terms.

E_real is the real-space Ewald pair sum over periodic images within r_c. The charge-charge term is undamped; the charge-dipole and dipole-dipole terms are Thole damped. For R = r_i - r_j + n C:

    U_ij = q_i q_j B0 + (q_i mu_j - q_j mu_i) . R B1t + (mu_i . mu_j) B1t
           - (mu_i . R)(mu_j . R) B2t

The damped functions are

    B_l^t = B_l - (2l - 1)!! (1 - lambda_{2l+1}) / R^(2l+1),  l = 1, 2, 3

with s = (a_i a_j)^(1/6), u = R / s and e = exp(-A u^3):

    1 - lambda_3 = e
    1 - lambda_5 = (1 + A u^3) e
    1 - lambda_7 = (1 + A u^3 + (3/5) A^2 u^6) e

They keep the recursion grad B_l^t = -R B_{l+1}^t of the undamped screened functions. Every derivative therefore takes the undamped form with B -> B^t.

Induced dipoles minimise U. U is quadratic in mu, so

    (diag(1/a) + H_real + H_pme) mu = -grad_mu (E_lr + E_real) at mu = 0,

where H_pme and H_real are the mu-mu Hessians of E_lr and E_real. Small systems
solve it densely (induced_dipoles); large ones by conjugate gradients with the PME
block applied matrix-free (induced_dipoles_cg), pinned to the dense solve.
"""
from __future__ import annotations

import math

import numpy as np

from . import pme as opme
from .ewald import _bl

THOLE_A = 0.39


def thole_b(r, s, alpha, A=THOLE_A):
    """B0 and the damped B1t, B2t, B3t at distances r for damping widths s
    (s = 0 or A = 0: no damping)."""
    B0, B1, B2, B3 = _bl(r, alpha, 3)
    with np.errstate(divide="ignore", invalid="ignore"):
        u3 = np.where(s > 0, (r / np.where(s > 0, s, 1.0)) ** 3, np.inf)
    au3 = A * u3
    e = np.where(np.isfinite(au3), np.exp(-np.where(np.isfinite(au3), au3, 0.0)), 0.0)
    au3 = np.where(np.isfinite(au3), au3, 0.0)
    m3 = e
    m5 = (1.0 + au3) * e
    m7 = (1.0 + au3 + 0.6 * au3 * au3) * e
    return (B0, B1 - m3 / r ** 3, B2 - 3.0 * m5 / r ** 5, B3 - 15.0 * m7 / r ** 7)


def _pairs(pos, box, rc):
    """All (i, j, R = r_i - r_j + n C) with 0 < |R| < rc over periodic images, in
    the order (i, j, image).  The centre atoms are taken in chunks, so memory stays
    bounded for large n; the chunks keep that order."""
    C = np.asarray(box, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    recip_len = np.linalg.norm(np.linalg.inv(C), axis=0)
    nmax = [int(math.ceil(rc * recip_len[a])) for a in range(3)]
    shifts = np.array([[i, j, k] for i in range(-nmax[0], nmax[0] + 1)
                       for j in range(-nmax[1], nmax[1] + 1)
                       for k in range(-nmax[2], nmax[2] + 1)], dtype=np.float64) @ C
    chunk = max(1, 4_000_000 // max(1, n * len(shifts)))
    out = [], [], [], []
    for s0 in range(0, n, chunk):
        R = (pos[s0:s0 + chunk, None, None, :] - pos[None, :, None, :]) + shifts[None, None, :, :]
        r = np.sqrt(np.einsum('ijsc,ijsc->ijs', R, R))
        ia, ja, sa = np.nonzero((r < rc) & (r > 1e-12))
        for lst, v in zip(out, (ia + s0, ja, R[ia, ja, sa], r[ia, ja, sa])):
            lst.append(v)
    if not out[0]:
        return (np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), np.zeros((0, 3)),
                np.zeros(0))
    return tuple(np.concatenate(v) for v in out)


def real_space(pos, q, mu, box, alpha, rc, pol, A=THOLE_A):
    """E_real and its gradients (dE/dr, dE/dmu); each ordered pair is visited, so
    the energy carries a factor 1/2."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    ia, ja, R, r = _pairs(pos, box, rc)
    s = (pol[ia] * pol[ja]) ** (1.0 / 6.0)
    B0, B1, B2, B3 = thole_b(r, s, alpha, A)
    B1u = _bl(r, alpha, 1)[1]                  # undamped B1 for the charge-charge force
    qi, qj, mi, mj = q[ia], q[ja], mu[ia], mu[ja]
    mir = np.einsum('pc,pc->p', mi, R)
    mjr = np.einsum('pc,pc->p', mj, R)
    mm = np.einsum('pc,pc->p', mi, mj)
    cross = qi * mjr - qj * mir
    U = qi * qj * B0 + cross * B1 + mm * B1 - mir * mjr * B2
    e = 0.5 * float(U.sum())
    gmu = np.zeros((n, 3))
    np.add.at(gmu, ia, (-qj * B1 - mjr * B2)[:, None] * R + B1[:, None] * mj)
    gR = ((-qi * qj * B1u - cross * B2 - mm * B2 + mir * mjr * B3)[:, None] * R
          + B1[:, None] * (qi[:, None] * mj - qj[:, None] * mi)
          - B2[:, None] * (mi * mjr[:, None] + mj * mir[:, None]))
    gpos = np.zeros((n, 3))
    np.add.at(gpos, ia, gR)
    return e, gpos, gmu


def real_mixed(pos, q, mu, box, alpha, rc, pol, v_pos, A=THOLE_A):
    """d/dmu (grad_r E_real . v_pos): the mu-r block of the real-space Hessian
    applied to a position cotangent."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    v = np.asarray(v_pos, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    ia, ja, R, r = _pairs(pos, box, rc)
    s = (pol[ia] * pol[ja]) ** (1.0 / 6.0)
    _, B1, B2, B3 = thole_b(r, s, alpha, A)
    w = v[ia] - v[ja]
    mj = mu[ja]
    qj = q[ja]
    rw = np.einsum('pc,pc->p', R, w)
    mjr = np.einsum('pc,pc->p', mj, R)
    mjw = np.einsum('pc,pc->p', mj, w)
    out = (-qj[:, None] * (w * B1[:, None] - R * (rw * B2)[:, None])
           - mj * (rw * B2)[:, None] - w * (mjr * B2)[:, None] - R * (mjw * B2)[:, None]
           + R * (rw * mjr * B3)[:, None])
    g = np.zeros((n, 3))
    np.add.at(g, ia, out)
    return g


def real_charge_grad(pos, q, mu, box, alpha, rc, pol, A=THOLE_A):
    """dE_real/dq (n,): differentiating the pair energy in q_i, the (i, j) and (j, i)
    visits give the same term, so with the factor 1/2
        dE/dq_i = sum_j [q_j B0 + (mu_j . R_ij) B1t]."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    ia, ja, R, r = _pairs(pos, box, rc)
    s = (pol[ia] * pol[ja]) ** (1.0 / 6.0)
    B0, B1, _, _ = thole_b(r, s, alpha, A)
    g = np.zeros(n)
    np.add.at(g, ia, q[ja] * B0 + np.einsum('pc,pc->p', mu[ja], R) * B1)
    return g


def real_hvp(pos, q, mu, box, alpha, rc, pol, v_pos=None, v_q=None, v_mu=None, A=THOLE_A):
    """The q and mu rows of the E_real Hessian in (r, q, mu) applied to the tangent
    (v_pos, v_q, v_mu): returns (h_q (n,), h_mu (n, 3)).

    E_real is bilinear in (q, mu), so the (q, mu) columns are the first-order
    gradients evaluated with charges v_q and dipoles v_mu.  The r column is the
    derivative of dE/dq_i and dE/dmu_i along w = v_i - v_j, with grad B0 = -R B1
    (undamped) and grad B_l^t = -R B_{l+1}^t:
        h_q  += -q_j B1 (R.w) + B1t (mu_j.w) - (mu_j.R) B2t (R.w)
        h_mu += the mu-r block of real_mixed."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    v = np.zeros((n, 3)) if v_pos is None else np.asarray(v_pos, dtype=np.float64)
    vq = np.zeros(n) if v_q is None else np.asarray(v_q, dtype=np.float64)
    vm = np.zeros((n, 3)) if v_mu is None else np.asarray(v_mu, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    ia, ja, R, r = _pairs(pos, box, rc)
    s = (pol[ia] * pol[ja]) ** (1.0 / 6.0)
    _, B1, B2, _ = thole_b(r, s, alpha, A)
    B1u = _bl(r, alpha, 1)[1]
    w = v[ia] - v[ja]
    rw = np.einsum('pc,pc->p', R, w)
    mjr = np.einsum('pc,pc->p', mu[ja], R)
    mjw = np.einsum('pc,pc->p', mu[ja], w)
    h_q = np.zeros(n)
    np.add.at(h_q, ia, -q[ja] * B1u * rw + B1 * mjw - mjr * B2 * rw)
    h_q += real_charge_grad(pos, vq, vm, box, alpha, rc, pol, A)
    h_mu = real_mixed(pos, q, mu, box, alpha, rc, pol, v, A)
    h_mu += real_space(pos, vq, vm, box, alpha, rc, pol, A)[2]
    return h_q, h_mu


def real_dipole_matrix(pos, box, alpha, rc, pol, A=THOLE_A):
    """Dense mu-mu Hessian of E_real, (3N, 3N)."""
    n = pos.shape[0]
    ia, ja, R, r = _pairs(np.asarray(pos, dtype=np.float64), box, rc)
    s = (np.asarray(pol)[ia] * np.asarray(pol)[ja]) ** (1.0 / 6.0)
    _, B1, B2, _ = thole_b(r, s, alpha, A)
    T = np.zeros((n, 3, n, 3))
    blk = B1[:, None, None] * np.eye(3)[None] - B2[:, None, None] * R[:, :, None] * R[:, None, :]
    np.add.at(T, (ia, slice(None), ja, slice(None)), blk)
    return T.reshape(3 * n, 3 * n)


def pme_dipole_matrix(pos, box, mesh, p, alpha, gamma=1.0):
    """Dense mu-mu Hessian of E_lr from Hessian-vector products with unit dipole
    cotangents (it does not depend on q or mu)."""
    n = pos.shape[0]
    zq = np.zeros(n)
    zmu = np.zeros((n, 3))
    H = np.zeros((3 * n, 3 * n))
    for k in range(3 * n):
        vm = np.zeros((n, 3))
        vm.reshape(-1)[k] = 1.0
        _, _, gmu = opme.hvp(pos, zq, zmu, box, mesh, p, alpha, None, None, vm, gamma)
        H[:, k] = gmu.reshape(-1)
    return H


def induced_dipoles(pos, q, box, mesh, p, alpha, rc, pol, A=THOLE_A, gamma=1.0):
    """Self-consistent dipoles by a dense linear solve (small systems)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.asarray(q, dtype=np.float64)
    zmu = np.zeros((n, 3))
    g_pme = opme.forward(pos, q, zmu, box, mesh, p, alpha, gamma).dE_dmu
    _, _, g_real = real_space(pos, q, zmu, box, alpha, rc, pol, A)
    b = -(g_pme + g_real).reshape(-1)
    Amat = (np.diag(np.repeat(1.0 / np.asarray(pol, dtype=np.float64), 3))
            + real_dipole_matrix(pos, box, alpha, rc, pol, A)
            + pme_dipole_matrix(pos, box, mesh, p, alpha, gamma))
    return np.linalg.solve(Amat, b).reshape(n, 3)


def real_dipole_sparse(pos, box, alpha, rc, pol, A=THOLE_A):
    """The matrix of real_dipole_matrix in sparse (CSR) form, for systems too large
    for the dense one: the same 3x3 pair blocks, duplicates summed."""
    import scipy.sparse as sp
    n = pos.shape[0]
    ia, ja, R, r = _pairs(np.asarray(pos, dtype=np.float64), box, rc)
    s = (np.asarray(pol)[ia] * np.asarray(pol)[ja]) ** (1.0 / 6.0)
    _, B1, B2, _ = thole_b(r, s, alpha, A)
    blk = B1[:, None, None] * np.eye(3)[None] - B2[:, None, None] * R[:, :, None] * R[:, None, :]
    k = np.arange(3)
    rows = (3 * ia)[:, None, None] + k[None, :, None] + 0 * k[None, None, :]
    cols = (3 * ja)[:, None, None] + 0 * k[None, :, None] + k[None, None, :]
    return sp.coo_matrix((blk.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(3 * n, 3 * n)).tocsr()


def induced_dipoles_cg(pos, q, box, mesh, p, alpha, rc, pol, A=THOLE_A, gamma=1.0,
                       tol=1e-12, max_iter=5000):
    """Self-consistent dipoles of the linear system of induced_dipoles, solved by
    plain conjugate gradients (Hestenes-Stiefel, no preconditioner) for systems too
    large for the dense matrix.  The PME block is applied matrix-free as the mu row
    of the E_lr Hessian-vector product with a dipole tangent (it is independent of
    q and mu, so it is taken at zero), the real-space block as the sparse matrix of
    real_dipole_sparse.  Stops once |b - A mu| <= tol |b|.  Returns (mu, iterations)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.asarray(q, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    zq = np.zeros(n)
    zmu = np.zeros((n, 3))
    g_pme = opme.forward(pos, q, zmu, box, mesh, p, alpha, gamma).dE_dmu
    _, _, g_real = real_space(pos, q, zmu, box, alpha, rc, pol, A)
    b = -(g_pme + g_real).reshape(-1)
    T = real_dipole_sparse(pos, box, alpha, rc, pol, A)
    d = np.repeat(1.0 / pol, 3)

    def apply(v):
        _, _, h = opme.hvp(pos, zq, zmu, box, mesh, p, alpha, None, None, v.reshape(n, 3), gamma)
        return d * v + T @ v + h.reshape(-1)

    x = np.zeros(3 * n)
    r = b.copy()
    s = r.copy()
    rr = float(r @ r)
    stop = tol * math.sqrt(float(b @ b))
    it = 0
    while math.sqrt(rr) > stop:
        if it == max_iter:
            raise RuntimeError(f"CG did not converge in {max_iter} iterations")
        As = apply(s)
        a = rr / float(s @ As)
        x += a * s
        r -= a * As
        rr_new = float(r @ r)
        s = r + (rr_new / rr) * s
        rr = rr_new
        it += 1
    return x.reshape(n, 3), it


def model(pos, q, mu, box, mesh, p, alpha, rc, pol, A=THOLE_A, gamma=1.0):
    """U(mu) and its gradients (dU/dr, dU/dmu) at the given dipoles."""
    pos = np.asarray(pos, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    f = opme.forward(pos, q, mu, box, mesh, p, alpha, gamma)
    er, gr_pos, gr_mu = real_space(pos, q, mu, box, alpha, rc, pol, A)
    u = f.energy + er + float(np.sum(np.sum(mu * mu, axis=1) / (2.0 * pol)))
    return u, f.dE_dpos + gr_pos, f.dE_dmu + gr_mu + mu / pol[:, None]


def model_grads(pos, q, mu, box, mesh, p, alpha, rc, pol, A=THOLE_A, gamma=1.0):
    """U and its gradients in all three inputs: (U, dU/dr, dU/dq, dU/dmu)."""
    pos = np.asarray(pos, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.float64)
    f = opme.forward(pos, q, mu, box, mesh, p, alpha, gamma)
    er, gr_pos, gr_mu = real_space(pos, q, mu, box, alpha, rc, pol, A)
    gr_q = real_charge_grad(pos, q, mu, box, alpha, rc, pol, A)
    u = f.energy + er + float(np.sum(np.sum(mu * mu, axis=1) / (2.0 * pol)))
    return u, f.dE_dpos + gr_pos, f.dE_dq + gr_q, f.dE_dmu + gr_mu + mu / pol[:, None]


def model_hvp(pos, q, mu, box, mesh, p, alpha, rc, pol, v_pos=None, v_q=None, v_mu=None,
              A=THOLE_A, gamma=1.0):
    """The q and mu rows of the Hessian of U (E_lr + E_real + polarization) in
    (r, q, mu) applied to (v_pos, v_q, v_mu): returns (h_q, h_mu)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    pol = np.asarray(pol, dtype=np.float64)
    vm = np.zeros((n, 3)) if v_mu is None else np.asarray(v_mu, dtype=np.float64)
    _, l_q, l_mu = opme.hvp(pos, q, mu, box, mesh, p, alpha, v_pos, v_q, v_mu, gamma)
    r_q, r_mu = real_hvp(pos, q, mu, box, alpha, rc, pol, v_pos, v_q, v_mu, A)
    return l_q + r_q, l_mu + r_mu + vm / pol[:, None]
