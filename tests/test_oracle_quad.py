"""Pins of the oracle's quadrupole channel (oracle/quad.py; CPU only), each against
something other than the formula it implements:

* a point multipole is the limit of a cluster of point charges with the same
  moments: the PME density and the explicit Ewald reciprocal energy of the
  quadrupoles are those of charge clusters (the pinned charge-only paths) as the
  cluster shrinks, and the closed-form self terms are the limit of the direct
  double sum of the screened kernel erf(a r)/r over the cluster;
* Theta = 0 gives the charge + dipole oracle exactly;
* the energy is invariant under a rotation of cell, positions, dipoles and second
  moments together (Theta -> R Theta R^T), which fails for a transposed mesh
  Jacobian in Q = J Theta J^T;
* every gradient matches central differences of the oracle's own energy;
* the PME result converges to the explicit Ewald sum as the mesh is refined.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import synth
from oracle import ewald, pme, quad


def _cluster(pos, q, mu, theta, h):
    """Point charges with, per atom, total charge q, first moment mu and second
    moment Theta (sum q r r^T), symmetric under inversion (no third moment from
    Theta)."""
    P, Q = [], []
    e = np.eye(3)
    for r, qi, mi, ti in zip(pos, q, mu, quad.theta_matrix(theta)):
        P.append(r)
        Q.append(qi)
        for a in range(3):
            for s in (1.0, -1.0):                        # dipole pair
                P.append(r + s * h * e[a])
                Q.append(s * mi[a] / (2.0 * h))
            c = ti[a, a] / (2.0 * h * h)                 # diagonal: +c, -2c, +c
            P += [r + h * e[a], r - h * e[a], r]
            Q += [c, c, -2.0 * c]
        for a, b in ((0, 1), (0, 2), (1, 2)):
            c = ti[a, b] / (4.0 * h * h)                 # off-diagonal: square of +-c
            for u, sg in ((e[a] + e[b], 1.0), (e[a] - e[b], -1.0)):
                P += [r + h * u, r - h * u]
                Q += [sg * c, sg * c]
    return np.array(P), np.array(Q)


def _frame(n, seed, L=11.0):
    rng = np.random.default_rng(seed)
    box = np.array([[L, 0.4, -0.3], [0.6, L + 0.5, 0.2], [-0.5, 0.7, L - 0.4]])
    pos = rng.uniform(0, 1, (n, 3)) @ box
    q = rng.normal(0, 1, n)
    q -= q.mean()
    mu = rng.normal(0, 0.3, (n, 3))
    th = synth.random_quadrupoles(n, seed + 100)
    return pos, q, mu, th, box


def test_cluster_moments():
    pos, q, mu, th, _ = _frame(3, 1)
    P, Q = _cluster(pos[:1], q[:1], mu[:1], th[:1], 0.1)
    d = P - pos[0]
    assert abs(Q.sum() - q[0]) < 1e-12
    assert np.allclose(Q @ d, mu[0], atol=1e-12)
    assert np.allclose(np.einsum('j,ja,jb->ab', Q, d, d), quad.theta_matrix(th[:1])[0], atol=1e-12)


@pytest.mark.parametrize("p", [4, 5, 6])
def test_density_is_the_charge_cluster_limit(p):
    pos, q, mu, th, box = _frame(12, 2 + p)
    mesh = (12, 13, 11)
    rho = quad.density(pos, q, mu, th, box, mesh, p)
    ref = {}
    for h in (2e-3, 1e-3):
        P, Q = _cluster(pos, q, mu, th, h)
        ref[h] = pme.density(P, Q, None, box, mesh, p)
    extra = (4.0 * ref[1e-3] - ref[2e-3]) / 3.0
    assert np.abs(extra - rho).max() <= 1e-7 * np.abs(rho).max()
    # the quadrupole part alone is not negligible
    rho0 = quad.density(pos, q, mu, None, box, mesh, p)
    assert np.abs(rho - rho0).max() > 0.1 * np.abs(rho).max()


def test_ewald_structure_factor_is_the_charge_cluster_limit():
    pos, q, mu, th, box = _frame(6, 3)
    th = 3.0 * th
    a, kc = 0.45, 4.0
    got = quad.ewald_long_range(pos, q, mu, th, box, a, kc=kc).e_recip
    e = {}
    for h in (2e-3, 1e-3):
        P, Q = _cluster(pos, q, mu, th, h)
        e[h] = ewald._recip_space(P, Q, np.zeros((len(Q), 3)), box, a, kc, False)[0]
    extra = (4.0 * e[1e-3] - e[2e-3]) / 3.0
    assert abs(extra - got) <= 1e-8 * abs(got)
    e0 = quad.ewald_long_range(pos, q, mu, None, box, a, kc=kc).e_recip
    assert abs(got - e0) > 0.05 * abs(got)


def _cluster_self(P, Q, a):
    """(1/2) sum_jk q_j q_k erf(a r_jk)/r_jk, the r = 0 terms 2a/sqrt(pi)."""
    d = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=2)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(d > 0, erf(a * np.where(d > 0, d, 1.0)) / np.where(d > 0, d, 1.0),
                     2.0 * a / math.sqrt(math.pi))
    return 0.5 * float(Q @ f @ Q)


@pytest.mark.parametrize("part", ["theta", "mu", "q-theta cross"])
def test_self_terms_are_the_cluster_limit(part):
    rng = np.random.default_rng(11)
    a = 0.4
    th = rng.normal(0, 0.4, (1, 6))
    mu = rng.normal(0, 0.4, (1, 3))
    q = np.array([0.8])
    z3, z1, z6 = np.zeros((1, 3)), np.zeros(1), np.zeros((1, 6))
    pos = np.zeros((1, 3))

    def si(qq, mm, tt):
        v = {}
        for h in (0.04, 0.02):
            P, Q = _cluster(pos, qq, mm, tt, h)
            v[h] = _cluster_self(P, Q, a)
        return (4.0 * v[0.02] - v[0.04]) / 3.0

    e_q, e_mu, e_th = quad.self_energy(q, mu, th, a)
    if part == "theta":
        got, want = -si(z1, z3, th), quad.self_energy(z1, z3, th, a)[2]
    elif part == "mu":
        got, want = -si(z1, mu, z6), e_mu
    else:
        got = -(si(q, z3, th) - si(q, z3, z6) - si(z1, z3, th))
        want = e_th - quad.self_energy(z1, z3, th, a)[2]
    assert abs(got - want) <= 1e-6 * abs(want)


def test_theta_zero_is_the_charge_dipole_oracle():
    pos, q, mu, _, box = _frame(15, 4)
    mesh, p, a = (12, 12, 12), 5, 0.4
    r = quad.forward(pos, q, mu, None, box, mesh, p, a, prefactor=1.3)
    s = pme.forward(pos, q, mu, box, mesh, p, a, prefactor=1.3)
    assert abs(r.energy - s.energy) <= 1e-13 * abs(s.energy)
    for x, y in ((r.dE_dpos, s.dE_dpos), (r.dE_dq, s.dE_dq), (r.dE_dmu, s.dE_dmu)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()
    ew = quad.ewald_long_range(pos, q, mu, None, box, a)
    e0, gp, gq, gm = ewald.ewald_long_range(pos, q, mu, box, a)
    assert abs(ew.energy - e0) <= 1e-12 * abs(e0)
    assert np.abs(ew.dE_dpos - gp).max() <= 1e-10 * np.abs(gp).max()


def _rot(seed):
    rng = np.random.default_rng(seed)
    Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return Rm


def test_rotation_invariance():
    pos, q, mu, th, box = _frame(14, 5)
    mesh, p, a = (12, 14, 13), 6, 0.4
    R = _rot(3)
    T = quad.theta_matrix(th)
    Tr = np.einsum('ab,nbc,dc->nad', R, T, R)
    thr = np.stack([Tr[:, i, j] for i, j in quad.PAIRS], axis=1)
    r0 = quad.forward(pos, q, mu, th, box, mesh, p, a)
    r1 = quad.forward(pos @ R.T, q, mu @ R.T, thr, box @ R.T, mesh, p, a)
    assert abs(r1.energy - r0.energy) <= 1e-12 * abs(r0.energy)
    assert np.abs(r1.dE_dpos - r0.dE_dpos @ R.T).max() <= 1e-10 * np.abs(r0.dE_dpos).max()
    # and a transposed Jacobian (J^T Theta J) would break it
    J = pme.jacobian(box, mesh)
    assert np.abs(J - J.T).max() > 1e-3


def _fd(fun, x, h):
    g = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        g[idx] = (fun(xp) - fun(xm)) / (2.0 * h)
    return g


def test_pme_gradients_finite_difference():
    pos, q, mu, th, box = _frame(8, 6)
    mesh, p, a = (10, 11, 12), 5, 0.45
    r = quad.forward(pos, q, mu, th, box, mesh, p, a, prefactor=1.7)
    E = lambda P=pos, Q=q, M=mu, T=th: quad.energy(P, Q, M, T, box, mesh, p, a, prefactor=1.7)
    checks = [(r.dE_dtheta, _fd(lambda x: E(T=x), th, 1e-5)),
              (r.dE_dpos, _fd(lambda x: E(P=x), pos, 1e-5)),
              (r.dE_dq, _fd(lambda x: E(Q=x), q, 1e-5)),
              (r.dE_dmu, _fd(lambda x: E(M=x), mu, 1e-5))]
    for got, fd in checks:
        assert np.abs(got - fd).max() <= 1e-7 * np.abs(fd).max()


def test_ewald_gradients_finite_difference():
    pos, q, mu, th, box = _frame(5, 7)
    a, kc = 0.45, 3.5
    r = quad.ewald_long_range(pos, q, mu, th, box, a, kc=kc)
    E = lambda P=pos, Q=q, M=mu, T=th: quad.ewald_long_range(P, Q, M, T, box, a, kc=kc).energy
    checks = [(r.dE_dtheta, _fd(lambda x: E(T=x), th, 1e-5)),
              (r.dE_dpos, _fd(lambda x: E(P=x), pos, 1e-5)),
              (r.dE_dq, _fd(lambda x: E(Q=x), q, 1e-5)),
              (r.dE_dmu, _fd(lambda x: E(M=x), mu, 1e-5))]
    for got, fd in checks:
        assert np.abs(got - fd).max() <= 1e-7 * np.abs(fd).max()


def test_pme_converges_to_ewald():
    pos, q, mu, th, box = _frame(10, 8, L=9.0)
    a = 0.4
    ew = quad.ewald_long_range(pos, q, mu, th, box, a)
    errs = []
    for p, spacing in [(5, 1.0), (6, 0.6), (7, 0.4)]:
        mesh = pme.mesh_dims(box, spacing, "smooth")
        r = quad.forward(pos, q, mu, th, box, mesh, p, a)
        errs.append((abs(r.energy - ew.energy) / abs(ew.energy),
                     np.abs(r.dE_dpos - ew.dE_dpos).max() / np.abs(ew.dE_dpos).max(),
                     np.abs(r.dE_dtheta - ew.dE_dtheta).max() / np.abs(ew.dE_dtheta).max()))
    for k in range(3):
        assert errs[0][k] > errs[1][k] > errs[2][k]
    assert max(errs[-1]) < 1e-6
