"""Pins of the oracle's optimal influence function (the alternative to the
sinc^(-2 gamma p) deconvolution; CPU only):

* restricted to the m = 0 alias it is G / U^2, the gamma = 1 deconvolution;
* it is even in f and, in a cubic cell, invariant under axis permutations;
* the aliases beyond |m| = 1 change it by less than 1e-3 where it matters (the
  truncation to m in {-1, 0, 1}^3 the library uses);
* on coarse meshes its forces are closer to the explicit Ewald forces than those
  of the deconvolution (what an optimal influence function is for), averaged over
  random configurations, and both converge to Ewald as the mesh is refined.  Its
  energies carry a mesh self-energy offset that the continuum self terms of the
  method do not remove, so the energy is not pinned against Ewald here.
"""
import numpy as np
import pytest

import synth
from oracle import ewald, pme


def _rms(a):
    return float(np.sqrt(np.mean(np.square(a))))


def test_m0_restriction_is_the_deconvolution():
    box = np.array([[12.0, 0.4, -0.3], [0.6, 11.0, 0.2], [-0.5, 0.7, 13.0]])
    mesh, p, a = (10, 12, 9), 5, 0.45
    g0 = pme.influence_optimal(box, mesh, p, a, m_max=0)
    g1 = pme.influence(box, mesh, p, a, gamma=1.0)
    assert np.allclose(g0, g1, rtol=1e-12, atol=0.0)


def test_symmetries():
    box = np.eye(3) * 14.0
    mesh, p, a = (12, 12, 12), 4, 0.5
    g = pme.influence_optimal(box, mesh, p, a)
    assert np.all(g >= 0.0) and g[0, 0, 0] == 0.0
    neg = [(-np.arange(n)) % n for n in mesh]
    gm = g[np.ix_(neg[0], neg[1], neg[2])]
    # even in f except on the Nyquist planes, where -(-N/2) is -N/2 again
    inner = np.ix_(*[np.r_[0:n // 2, n // 2 + 1:n] for n in mesh])
    assert np.allclose(g[inner], gm[inner], rtol=1e-12, atol=0.0)
    assert np.allclose(g, np.transpose(g, (1, 0, 2)), rtol=1e-12, atol=0.0)
    assert np.allclose(g, np.transpose(g, (2, 1, 0)), rtol=1e-12, atol=0.0)


def test_alias_truncation():
    box = np.eye(3) * 18.0
    mesh, p, a = (10, 10, 10), 4, 0.45
    g1 = pme.influence_optimal(box, mesh, p, a, m_max=1)
    g2 = pme.influence_optimal(box, mesh, p, a, m_max=2)
    big = g2 > 1e-6 * g2.max()
    assert np.max(np.abs(g1[big] - g2[big]) / g2[big]) < 1e-3


def test_forces_closer_to_ewald_on_coarse_meshes():
    errs = {1.0: [], "optimal": []}
    for seed in (1, 2, 3):
        f = synth.molten_box(200, seed)
        for a, M, p in [(0.45, 10, 4), (0.5, 12, 5), (0.4, 8, 4)]:
            _, gref, _, _ = ewald.ewald_long_range(f.pos, f.q, f.mu, f.box, a)
            for gam in errs:
                r = pme.forward(f.pos, f.q, f.mu, f.box, (M, M, M), p, a, gamma=gam)
                errs[gam].append(_rms(r.dE_dpos - gref) / _rms(gref))
    e_dec, e_opt = np.array(errs[1.0]), np.array(errs["optimal"])
    assert np.all(e_opt < e_dec)
    assert e_opt.mean() < 0.95 * e_dec.mean()


def test_converges_to_ewald():
    f = synth.molten_box(200, 4)
    a = 0.35
    _, gref, _, gm = ewald.ewald_long_range(f.pos, f.q, f.mu, f.box, a)
    prev = None
    for p, M in [(4, 12), (5, 20), (6, 32)]:
        r = pme.forward(f.pos, f.q, f.mu, f.box, (M, M, M), p, a, gamma="optimal")
        err = (_rms(r.dE_dpos - gref) / _rms(gref), _rms(r.dE_dmu - gm) / _rms(gm))
        if prev is not None:
            assert err[0] < prev[0] and err[1] < prev[1]
        prev = err
    assert prev[0] < 1e-5
