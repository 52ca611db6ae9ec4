"""Pins of the CPU particle-mesh oracle (CPU only).

* convergence to the explicit Ewald reciprocal + self energy and gradients as
  the mesh is refined and the order p is raised (the paper's claim that the
  deconvolved PME reproduces Ewald, Sec. 3.1), including the charge-dipole and
  dipole-dipole terms, which pins the dipole sign convention;
* the influence-correction ablation: gamma = 0 leaves a much larger error than
  gamma = 1 (Eq. influence and the Sec. 3.1 ablation);
* Eq. energy_recip equals (1/2V) sum_k g |rho~|^2 (unnormalised inverse);
* finite differences of the analytic gradient and of the Hessian-vector
  product, exact differences along q and mu, the Euler identity, Hessian
  symmetry;
* exact invariances: lattice and mesh-vector translation, inversion, cubic
  axis permutation.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ewald, pme


def _rms(a):
    return float(np.sqrt(np.mean(np.square(a))))


def test_converges_to_ewald_charges():
    f = synth.rocksalt()
    a = 0.3
    e_lr, g, _, _ = ewald.ewald_long_range(f.pos, f.q, None, f.box, a)
    errs = []
    for p, M in [(4, 16), (4, 32), (6, 32), (7, 48)]:
        r = pme.forward(f.pos, f.q, None, f.box, (M, M, M), p, a)
        errs.append((abs(r.energy - e_lr) / f.n, _rms(r.dE_dpos - g)))
    # monotone in mesh and order, and the finest case is at round-off level
    for (e0, f0), (e1, f1) in zip(errs, errs[1:]):
        assert e1 < e0 and f1 < f0
    assert errs[-1][0] < 1e-12 and errs[-1][1] < 1e-10


def test_converges_to_ewald_charges_and_dipoles():
    f = synth.molten_box(200, 1)
    a = 0.3
    e_lr, g, gq, gm = ewald.ewald_long_range(f.pos, f.q, f.mu, f.box, a)
    prev = None
    for p, M in [(6, 16), (6, 32), (7, 40)]:
        r = pme.forward(f.pos, f.q, f.mu, f.box, (M, M, M), p, a)
        err = (abs(r.energy - e_lr) / f.n, _rms(r.dE_dpos - g), _rms(r.dE_dq - gq),
               _rms(r.dE_dmu - gm))
        if prev is not None:
            assert all(e1 < e0 for e0, e1 in zip(prev, err))
        prev = err
    assert prev[0] < 1e-10 and max(prev[1:]) < 1e-8


def test_dipole_only_system_converges():
    # pure dipole-dipole electrostatics (no charges) against Ewald
    f = synth.molten_box(64, 9, L=14.0, mu_sigma=0.4)
    a = 0.35
    e_lr, g, _, gm = ewald.ewald_long_range(f.pos, None, f.mu, f.box, a)
    r = pme.forward(f.pos, None, f.mu, f.box, (48, 48, 48), 7, a)
    # the residual is the mesh self-interaction of each smeared dipole, which the
    # continuum self term leaves in (it oscillates with the mesh, at ~1e-8 here)
    assert r.energy == pytest.approx(e_lr, rel=1e-6)
    assert _rms(r.dE_dpos - g) < 1e-6 * _rms(g)
    assert _rms(r.dE_dmu - gm) < 1e-6 * _rms(gm)


def test_influence_ablation_gamma0_is_worse():
    f = synth.rocksalt()
    a = 0.3
    e_lr, g, _, _ = ewald.ewald_long_range(f.pos, f.q, None, f.box, a)
    for p, M in [(4, 32), (7, 48)]:
        r1 = pme.forward(f.pos, f.q, None, f.box, (M, M, M), p, a, gamma=1.0)
        r0 = pme.forward(f.pos, f.q, None, f.box, (M, M, M), p, a, gamma=0.0)
        assert abs(r0.energy - e_lr) > 100 * abs(r1.energy - e_lr)
        assert _rms(r0.dE_dpos - g) > 100 * _rms(r1.dE_dpos - g)


def test_energy_equals_spectral_sum_and_prefactor():
    f = synth.molten_box(100, 2, L=15.0)
    mesh, p, a = (16, 18, 20), 5, 0.4
    r = pme.forward(f.pos, f.q, f.mu, f.box, mesh, p, a)
    g = pme.influence(f.box, mesh, p, a)
    rt = np.fft.fftn(r.rho)
    V = abs(np.linalg.det(f.box))
    assert r.e_recip == pytest.approx(float(np.sum(g * np.abs(rt) ** 2)) / (2 * V), rel=1e-12)
    k = 14.3996454784
    r2 = pme.forward(f.pos, f.q, f.mu, f.box, mesh, p, a, prefactor=k)
    assert r2.energy == pytest.approx(k * r.energy, rel=1e-14)
    assert np.allclose(r2.dE_dpos, k * r.dE_dpos, rtol=1e-13, atol=0)


def _small():
    f = synth.molten_box(40, 3, L=12.0)
    return f, (f.box, (12, 12, 12), 6, 0.35)


def test_gradients_finite_difference():
    f, args = _small()
    r = pme.forward(f.pos, f.q, f.mu, *args)
    rng = np.random.default_rng(0)
    for _ in range(2):
        d = rng.normal(size=f.pos.shape)
        h = 1e-4
        ep = pme.energy(f.pos + h * d, f.q, f.mu, *args)
        em = pme.energy(f.pos - h * d, f.q, f.mu, *args)
        assert (ep - em) / (2 * h) == pytest.approx(np.sum(r.dE_dpos * d), rel=1e-7)
    dq = rng.normal(size=f.n)
    dm = rng.normal(size=(f.n, 3))
    eq = (pme.energy(f.pos, f.q + dq, f.mu, *args) - pme.energy(f.pos, f.q - dq, f.mu, *args)) / 2
    em = (pme.energy(f.pos, f.q, f.mu + dm, *args) - pme.energy(f.pos, f.q, f.mu - dm, *args)) / 2
    assert eq == pytest.approx(np.sum(r.dE_dq * dq), rel=1e-11)
    assert em == pytest.approx(np.sum(r.dE_dmu * dm), rel=1e-11)
    assert 2 * r.energy == pytest.approx(np.sum(f.q * r.dE_dq) + np.sum(f.mu * r.dE_dmu), rel=1e-12)


@pytest.mark.parametrize("p", [4, 5, 6, 7])
def test_hvp_finite_difference_and_symmetry(p):
    f, args = _small()
    args = (args[0], args[1], p, args[3])
    v = synth.random_cotangents(f.n, 5)
    hv = pme.hvp(f.pos, f.q, f.mu, *args, v_pos=v[0], v_q=v[1], v_mu=v[2])
    h = 1e-4

    def grad(s):
        r = pme.forward(f.pos + s * v[0], f.q + s * v[1], f.mu + s * v[2], *args)
        return r.dE_dpos, r.dE_dq, r.dE_dmu

    gp, gm = grad(h), grad(-h)
    for a, b, c in zip(hv, gp, gm):
        fd = (b - c) / (2 * h)
        assert np.max(np.abs(a - fd)) < 1e-6 * np.max(np.abs(fd))
    w = synth.random_cotangents(f.n, 9)
    hw = pme.hvp(f.pos, f.q, f.mu, *args, v_pos=w[0], v_q=w[1], v_mu=w[2])
    lhs = sum(np.sum(x * y) for x, y in zip(w, hv))
    rhs = sum(np.sum(x * y) for x, y in zip(v, hw))
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_hvp_force_loss_is_linear_in_q_mu():
    # with v_q = v_mu = 0 (a force loss) the (q, mu) outputs are linear in (q, mu);
    # the position output is quadratic, since the Hessian in r is
    f, args = _small()
    v = synth.random_cotangents(f.n, 2)[0]
    a = pme.hvp(f.pos, f.q, f.mu, *args, v_pos=v)
    b = pme.hvp(f.pos, 2.5 * f.q, 2.5 * f.mu, *args, v_pos=v)
    assert np.allclose(6.25 * a[0], b[0], rtol=1e-11, atol=1e-14)
    for x, y in zip(a[1:], b[1:]):
        assert np.allclose(2.5 * x, y, rtol=1e-11, atol=1e-14)


def test_exact_invariances():
    f = synth.molten_box(60, 4, L=13.0)
    mesh, p, a = (13, 13, 13), 6, 0.35
    r = pme.forward(f.pos, f.q, f.mu, f.box, mesh, p, a)
    # lattice translation of one atom and of all atoms
    shifted = f.pos.copy()
    shifted[3] += f.box[1]
    shifted -= 2 * f.box[2]
    r1 = pme.forward(shifted, f.q, f.mu, f.box, mesh, p, a)
    assert r1.energy == pytest.approx(r.energy, rel=1e-12)
    assert np.allclose(r1.dE_dpos, r.dE_dpos, atol=1e-11)
    # translation by a mesh vector a_x / N_x
    r2 = pme.forward(f.pos + f.box[0] / mesh[0], f.q, f.mu, f.box, mesh, p, a)
    assert r2.energy == pytest.approx(r.energy, rel=1e-12)
    assert np.allclose(r2.dE_dpos, r.dE_dpos, atol=1e-11)
    assert np.allclose(np.roll(r.rho, 1, axis=0), r2.rho, atol=1e-12)
    # inversion r -> -r, mu -> -mu (even p keeps the stencil symmetric)
    r3 = pme.forward(-f.pos, f.q, -f.mu, f.box, mesh, p, a)
    assert r3.energy == pytest.approx(r.energy, rel=1e-11)
    assert np.allclose(r3.dE_dpos, -r.dE_dpos, atol=1e-10)
    # cubic axis permutation (x, y, z) -> (y, z, x)
    perm = [1, 2, 0]
    r4 = pme.forward(f.pos[:, perm], f.q, f.mu[:, perm], f.box, mesh, p, a)
    assert r4.energy == pytest.approx(r.energy, rel=1e-12)
    assert np.allclose(r4.dE_dpos, r.dE_dpos[:, perm], atol=1e-11)


def test_triclinic_cell_against_ewald():
    f = synth.triclinic_cell()
    a = 0.45
    e_lr, g, gq, gm = ewald.ewald_long_range(f.pos, f.q, f.mu, f.box, a)
    mesh = pme.mesh_dims(f.box, 0.5, "smooth")
    r = pme.forward(f.pos, f.q, f.mu, f.box, mesh, 7, a)
    assert r.energy == pytest.approx(e_lr, rel=1e-7)
    assert _rms(r.dE_dpos - g) < 1e-5 * _rms(g)
    assert _rms(r.dE_dmu - gm) < 1e-5 * _rms(gm)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_low_orders_charge_energy_and_gradient(p):
    # p = 1, 2 have a.e. vanishing higher derivatives; q-gradients are still exact
    f, args = _small()
    args = (args[0], args[1], p, args[3])
    r = pme.forward(f.pos, f.q, None, *args)
    dq = np.random.default_rng(1).normal(size=f.n)
    eq = (pme.energy(f.pos, f.q + dq, None, *args) - pme.energy(f.pos, f.q - dq, None, *args)) / 2
    assert eq == pytest.approx(np.sum(r.dE_dq * dq), rel=1e-11)
