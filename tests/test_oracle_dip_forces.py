"""Pins of the oracle's conservative student forces (oracle/dip.py: position_vjp,
conservative_forces; CPU only):

* the radial derivative against central differences of the radial basis;
* the position vector-Jacobian product against central differences of
  sum_i u_i . mu_i(r), the dipole head evaluated on moved positions;
* it sums to zero over the atoms (the features depend on differences only);
* the conservative force against central differences of the total energy
  U(r, mu_NN(r)) of the student model through PME.
"""
import numpy as np
import pytest

import synth
from oracle import dip as odip
from oracle import pol as opol


def _sys(n=12, L=12.0, seed=4):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return pos, q, np.eye(3) * L, np.where(q > 0, 0.15, 3.5)


def _mu(theta, pos, q, box, rc):
    x, V = odip.features(pos, q, box, rc)
    return odip.dipoles(theta, x, V)[0]


def test_radial_derivative():
    r = np.linspace(0.3, 4.99, 57)
    h = 1e-6
    fd = (odip.radial(r + h, 5.0) - odip.radial(r - h, 5.0)) / (2 * h)
    assert np.abs(odip.radial_derivative(r, 5.0) - fd).max() <= 1e-7 * np.abs(fd).max()
    # zero at and beyond the cutoff
    assert np.abs(odip.radial_derivative(np.array([5.0, 5.5]), 5.0)).max() == 0.0


def test_position_vjp_finite_difference():
    pos, q, box, _ = _sys(n=14, seed=5)
    rc = 5.0
    theta = synth.mlp_init(3, last_scale=1.0)
    u = np.random.default_rng(2).normal(size=(len(q), 3))
    g = odip.position_vjp(theta, pos, q, box, rc, u)
    h = 1e-5
    fd = np.zeros_like(pos)
    for j in range(len(q)):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, d] += h
            pm[j, d] -= h
            fd[j, d] = (np.sum(u * _mu(theta, pp, q, box, rc))
                        - np.sum(u * _mu(theta, pm, q, box, rc))) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()
    assert np.abs(g.sum(axis=0)).max() <= 1e-12 * np.abs(g).max() * len(q)


@pytest.mark.slow
def test_conservative_force_is_minus_total_energy_gradient():
    pos, q, box, pol = _sys(n=8, seed=6)
    mesh, p, alpha, rc = (12, 12, 12), 5, 0.35, 5.5
    theta = synth.mlp_init(2, last_scale=1.0)
    F, U, mu = odip.conservative_forces(theta, pos, q, pol, box, mesh, p, alpha, rc, 5.0)

    def total(P):
        m = _mu(theta, P, q, box, 5.0)
        return opol.model(P, q, m, box, mesh, p, alpha, rc, pol)[0]

    h = 1e-5
    for j, d in [(0, 0), (3, 1), (5, 2), (7, 0)]:
        pp, pm = pos.copy(), pos.copy()
        pp[j, d] += h
        pm[j, d] -= h
        fd = -(total(pp) - total(pm)) / (2 * h)
        assert abs(F[j, d] - fd) <= 1e-6 * np.abs(F).max(), (j, d, F[j, d], fd)
    # and it differs from the Hellmann-Feynman force (the dipole head moves with r)
    _, dUdr, _ = opol.model(pos, q, mu, box, mesh, p, alpha, rc, pol)
    assert np.abs(F + dUdr).max() > 1e-3 * np.abs(F).max()
