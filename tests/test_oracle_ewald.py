"""Pins of the explicit-Ewald oracle against closed forms and invariants (CPU).

* rock-salt Madelung energy for several splitting parameters;
* two opposite charges in a cubic box: -1/d - 2 pi d^2/(3 L^3) - c4 d^4/L^5,
  the tin-foil surface term plus the cubic l = 4 lattice sum c4 (computed here
  by brute force over the integer lattice);
* a single point dipole in a cubic box: exactly -2 pi |mu|^2 / (3 L^3);
* independence of the total energy from alpha, zero net force, finite
  differences of the analytic gradients.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import ewald

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MADELUNG = float([l for l in open(os.path.join(GOLDEN, "madelung.txt"))
                  if not l.startswith("#")][0])


@pytest.mark.parametrize("alpha", [0.2, 0.3, 0.5, 1.0])
def test_madelung_rocksalt(alpha):
    f = synth.rocksalt(displaced=False)
    r = ewald.ewald(f.pos, f.q, None, f.box, alpha)
    expect = -32 * MADELUNG / (synth.ROCKSALT_A / 2)
    assert r.energy == pytest.approx(expect, rel=1e-10)
    assert np.max(np.abs(r.dE_dpos)) < 1e-10


def _c4(nmax=40):
    """sum_{n != 0} P_4(n_x/|n|) / |n|^5 over the simple cubic lattice (absolutely convergent)."""
    r = np.arange(-nmax, nmax + 1, dtype=float)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    R2 = X * X + Y * Y + Z * Z
    R2[nmax, nmax, nmax] = 1.0
    c = X * X / R2
    p4 = (35 * c * c - 30 * c + 3) / 8
    term = p4 / R2 ** 2.5
    term[nmax, nmax, nmax] = 0.0
    return float(term.sum())


@pytest.mark.parametrize("L", [40.0, 60.0])
def test_charged_dimer_closed_form(L):
    d = 3.0
    pos = np.array([[4.0, 5.0, 6.0], [4.0 + d, 5.0, 6.0]])
    q = np.array([1.0, -1.0])
    r = ewald.ewald(pos, q, None, np.eye(3) * L, 0.3)
    c4 = _c4()
    expect = -1 / d - 2 * math.pi * d * d / (3 * L ** 3) - c4 * d ** 4 / L ** 5
    assert r.energy == pytest.approx(expect, abs=5e-9)
    # dE/dd = 1/d^2 - 4 pi d/(3 L^3) - 4 c4 d^3 / L^5 acts on the second atom along x
    dEdd = 1 / d ** 2 - 4 * math.pi * d / (3 * L ** 3) - 4 * c4 * d ** 3 / L ** 5
    assert r.dE_dpos[1, 0] == pytest.approx(dEdd, abs=1e-8)
    assert r.dE_dpos[0, 0] == pytest.approx(-dEdd, abs=1e-8)


@pytest.mark.parametrize("alpha", [0.25, 0.4])
def test_single_dipole_closed_form(alpha):
    L = 20.0
    mu = np.array([[0.1, 0.0, 0.0]])
    r = ewald.ewald(np.array([[1.0, 2.0, 3.0]]), np.zeros(1), mu, np.eye(3) * L, alpha)
    expect = -2 * math.pi * 0.01 / (3 * L ** 3)
    assert r.energy == pytest.approx(expect, rel=1e-9)
    # dE/dmu = -4 pi mu / (3 L^3)
    assert np.allclose(r.dE_dmu, -4 * math.pi * mu / (3 * L ** 3), atol=1e-13)


def _random_system(n=8, seed=11, L=9.0, charges=True, dipoles=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (n, 3))
    q = rng.normal(0, 1, n) if charges else np.zeros(n)
    q -= q.mean()
    mu = rng.normal(0, 0.3, (n, 3)) if dipoles else np.zeros((n, 3))
    return pos, q, mu, np.eye(3) * L


def test_alpha_independence_and_net_force():
    pos, q, mu, box = _random_system()
    ref = ewald.ewald(pos, q, mu, box, 0.35)
    for a in (0.3, 0.45, 0.6):
        r = ewald.ewald(pos, q, mu, box, a)
        assert r.energy == pytest.approx(ref.energy, rel=1e-10, abs=1e-12)
        assert np.allclose(r.dE_dpos, ref.dE_dpos, atol=1e-9)
        assert np.allclose(r.dE_dq, ref.dE_dq, atol=1e-9)
        assert np.allclose(r.dE_dmu, ref.dE_dmu, atol=1e-9)
    scale = np.max(np.abs(ref.dE_dpos))
    assert np.max(np.abs(ref.dE_dpos.sum(axis=0))) < 1e-10 * max(1.0, scale)


def test_alpha_independence_triclinic_non_neutral_background():
    f = synth.triclinic_cell()
    q = f.q + 0.3                              # net charge 2.4 e
    e = [ewald.ewald(f.pos, q, f.mu, f.box, a, background=True).energy for a in (0.35, 0.5)]
    assert e[0] == pytest.approx(e[1], rel=1e-10)


def test_finite_difference_gradients():
    pos, q, mu, box = _random_system(n=6, seed=4)
    a = 0.4
    r = ewald.ewald(pos, q, mu, box, a)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(3):
        d = rng.normal(size=pos.shape)
        ep = ewald.ewald(pos + h * d, q, mu, box, a, want_grad=False).energy
        em = ewald.ewald(pos - h * d, q, mu, box, a, want_grad=False).energy
        assert (ep - em) / (2 * h) == pytest.approx(np.sum(r.dE_dpos * d), rel=1e-7, abs=1e-9)
    # E is a homogeneous quadratic in (q, mu): central differences are exact at any step
    dq = rng.normal(size=q.shape)
    dm = rng.normal(size=mu.shape)
    eq = (ewald.ewald(pos, q + dq, mu, box, a, want_grad=False).energy
          - ewald.ewald(pos, q - dq, mu, box, a, want_grad=False).energy) / 2
    em_ = (ewald.ewald(pos, q, mu + dm, box, a, want_grad=False).energy
           - ewald.ewald(pos, q, mu - dm, box, a, want_grad=False).energy) / 2
    assert eq == pytest.approx(np.sum(r.dE_dq * dq), rel=1e-10)
    assert em_ == pytest.approx(np.sum(r.dE_dmu * dm), rel=1e-10)
    # Euler identity for a homogeneous quadratic
    assert 2 * r.energy == pytest.approx(np.sum(q * r.dE_dq) + np.sum(mu * r.dE_dmu), rel=1e-10)
