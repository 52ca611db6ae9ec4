"""Pins of the polarizable-model oracle (oracle/pol.py), all in FP64 on the CPU.

* The damped B_l^t keep the recursion d/dR B_l^t = -R B_{l+1}^t. A wrong damping polynomial breaks it.
* Without polarizability the damping vanishes, and the real-space sum equals the explicit-Ewald real-space sum. That sum is pinned by the Madelung constant and by alpha-independence.
* Analytic gradients match central differences: positions and dipoles, plus the mixed mu-r block.
* The dense solve is a stationary point and a minimum of U. It is linear in the charges.
"""
import numpy as np
import pytest

from oracle import ewald as oew
from oracle import pol as opol
from oracle.ewald import _bl

pytestmark = []


def _system(n=12, L=12.0, seed=3):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    mu = rng.normal(0, 0.2, (n, 3))
    pol = np.where(q > 0, 0.15, 3.5)
    return pos, q, mu, np.eye(3) * L, pol


def test_thole_recursion_finite_difference():
    rng = np.random.default_rng(0)
    r = rng.uniform(1.0, 6.0, 20)
    s = rng.uniform(0.6, 1.6, 20)
    h = 1e-6
    Bp = opol.thole_b(r + h, s, 0.3)
    Bm = opol.thole_b(r - h, s, 0.3)
    B = opol.thole_b(r, s, 0.3)
    for l in (1, 2):
        d = (Bp[l] - Bm[l]) / (2 * h)
        np.testing.assert_allclose(d, -r * B[l + 1], rtol=1e-7, atol=1e-12)
    # the charge function is undamped: d/dR B0 = -R B1 (undamped)
    d0 = (Bp[0] - Bm[0]) / (2 * h)
    np.testing.assert_allclose(d0, -r * _bl(r, 0.3, 1)[1], rtol=1e-7)


def test_damping_vanishes_without_polarizability():
    pos, q, mu, box, pol = _system()
    rc = 5.5
    e, gpos, gmu = opol.real_space(pos, q, mu, box, 0.35, rc, np.full(len(q), 1e-30))
    e0, gpos0, _, gmu0 = oew._real_space(pos, q, mu, box, 0.35, rc, True)
    assert abs(e - e0) <= 1e-12 * abs(e0)
    np.testing.assert_allclose(gpos, gpos0, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gmu, gmu0, rtol=1e-10, atol=1e-12)
    # and with polarizability the damping changes the dipole terms only
    e1, _, _ = opol.real_space(pos, q, None, box, 0.35, rc, pol)
    e2, _, _ = opol.real_space(pos, q, None, box, 0.35, rc, np.full(len(q), 1e-30))
    assert abs(e1 - e2) <= 1e-12 * abs(e2)


def test_real_space_gradients_finite_difference():
    pos, q, mu, box, pol = _system(n=8, seed=5)
    rc = 5.5
    _, gpos, gmu = opol.real_space(pos, q, mu, box, 0.35, rc, pol)
    h = 1e-5
    for i in range(3):
        for c in range(3):
            dp = np.zeros_like(pos)
            dp[i, c] = h
            ep = opol.real_space(pos + dp, q, mu, box, 0.35, rc, pol)[0]
            em = opol.real_space(pos - dp, q, mu, box, 0.35, rc, pol)[0]
            assert abs((ep - em) / (2 * h) - gpos[i, c]) < 1e-6 * (1 + abs(gpos[i, c]))
            # E is quadratic in mu: central differences are exact up to rounding
            ep = opol.real_space(pos, q, mu + dp, box, 0.35, rc, pol)[0]
            em = opol.real_space(pos, q, mu - dp, box, 0.35, rc, pol)[0]
            assert abs((ep - em) / (2 * h) - gmu[i, c]) < 1e-7 * (1 + abs(gmu[i, c]))


def test_real_mixed_block_finite_difference():
    pos, q, mu, box, pol = _system(n=8, seed=6)
    rc = 5.5
    v = np.random.default_rng(1).normal(0, 1, pos.shape)
    g = opol.real_mixed(pos, q, mu, box, 0.35, rc, pol, v)
    h = 1e-5
    gp = opol.real_space(pos + h * v, q, mu, box, 0.35, rc, pol)[2]
    gm = opol.real_space(pos - h * v, q, mu, box, 0.35, rc, pol)[2]
    np.testing.assert_allclose(g, (gp - gm) / (2 * h), rtol=1e-6, atol=1e-8)


def test_dipole_matrices_symmetric_and_consistent():
    pos, q, mu, box, pol = _system(n=6, seed=7)
    T = opol.real_dipole_matrix(pos, box, 0.35, 5.5, pol)
    np.testing.assert_allclose(T, T.T, atol=1e-12)
    # T mu equals the dipole part of the real-space mu-gradient
    _, _, g1 = opol.real_space(pos, None, mu, box, 0.35, 5.5, pol)
    np.testing.assert_allclose(T @ mu.reshape(-1), g1.reshape(-1), rtol=1e-10, atol=1e-12)
    H = opol.pme_dipole_matrix(pos, box, (12, 12, 12), 5, 0.35)
    np.testing.assert_allclose(H, H.T, atol=1e-10)


@pytest.mark.slow
def test_scf_stationary_minimum_and_linear():
    pos, q, _, box, pol = _system(n=8, seed=8)
    mesh, p, a, rc = (12, 12, 12), 5, 0.35, 5.5
    mu = opol.induced_dipoles(pos, q, box, mesh, p, a, rc, pol)
    u0, _, gmu = opol.model(pos, q, mu, box, mesh, p, a, rc, pol)
    assert np.abs(gmu).max() < 1e-9
    rng = np.random.default_rng(2)
    for _ in range(3):
        d = rng.normal(0, 0.05, mu.shape)
        assert opol.model(pos, q, mu + d, box, mesh, p, a, rc, pol)[0] > u0
    mu2 = opol.induced_dipoles(pos, 2 * q, box, mesh, p, a, rc, pol)
    np.testing.assert_allclose(mu2, 2 * mu, rtol=1e-9, atol=1e-12)


def test_sparse_real_dipole_matrix_equals_dense():
    pos, q, mu, box, pol = _system(n=9, seed=11)
    T = opol.real_dipole_matrix(pos, box, 0.35, 5.5, pol)
    S = opol.real_dipole_sparse(pos, box, 0.35, 5.5, pol).toarray()
    np.testing.assert_allclose(S, T, rtol=1e-13, atol=1e-14)


@pytest.mark.slow
def test_cg_solve_equals_dense_solve():
    """The matrix-free CG solve (used where the dense matrix does not fit) reaches
    the dense solve's dipoles, and they zero dU/dmu of the forward calls."""
    pos, q, _, box, pol = _system(n=10, seed=12)
    mesh, p, a, rc = (12, 12, 12), 5, 0.35, 5.5
    ref = opol.induced_dipoles(pos, q, box, mesh, p, a, rc, pol)
    mu, it = opol.induced_dipoles_cg(pos, q, box, mesh, p, a, rc, pol, tol=1e-13)
    assert 0 < it <= 3 * len(q) + 5
    np.testing.assert_allclose(mu, ref, rtol=1e-9, atol=1e-11)
    _, _, gmu = opol.model(pos, q, mu, box, mesh, p, a, rc, pol)
    assert np.abs(gmu).max() < 1e-9
