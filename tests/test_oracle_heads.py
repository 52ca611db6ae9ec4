"""Pins of the oracle's charge head and of training on conservative forces
(oracle/heads.py, and the real-space charge and Hessian rows of oracle/pol.py;
CPU only).

* dE_real/dq and dU/dq against central differences of the energies in q;
* the q and mu rows of the real-space and full-model Hessians against central
  differences of the first-order gradients along (v_pos, v_q, v_mu);
* the feature tangent against central differences of the features along v, and
  the feature transpose against the tangent (adjoint identity);
* the charge head: neutrality, translation invariance, the cubic symmetry of the
  cell, the zero-output special case, and its forward-mode derivative;
* reverse mode through the heads' dual evaluation against central differences
  in the parameters;
* the head channels of the force against central differences of u . mu(r) +
  c . q(r), and the conservative force against those of the total energy;
* the loss gradient, conservative and Hellmann-Feynman, against central
  differences of the loss in the parameters.
"""
import numpy as np
import pytest

import synth
from oracle import dip as odip
from oracle import heads as oh
from oracle import pol as opol


def _sys(n=12, L=12.0, seed=4):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (n, 3))
    z = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return pos, z, np.eye(3) * L, np.where(z > 0, 0.15, 3.5)


def _params(seed=3):
    theta = synth.mlp_init(seed, last_scale=1.0)
    thq = synth.charge_head_init(seed + 1, last_scale=1.0, bias_scale=0.5)
    return theta, thq


def _cd(f, x0, d, h):
    return (f(x0 + h * d) - f(x0 - h * d)) / (2 * h)


def test_parameter_count():
    assert oh.NQPARAM == 64 * 34 + 64 + 64 == 2304
    assert synth.charge_head_init(0).size == oh.NQPARAM


def test_real_charge_gradient_finite_difference():
    pos, z, box, pol = _sys(n=10, seed=1)
    rng = np.random.default_rng(0)
    q = z + 0.2 * rng.normal(size=len(z))
    mu = 0.3 * rng.normal(size=(len(z), 3))
    alpha, rc = 0.35, 5.5
    g = opol.real_charge_grad(pos, q, mu, box, alpha, rc, pol)
    d = rng.normal(size=len(z))
    fd = _cd(lambda qq: opol.real_space(pos, qq, mu, box, alpha, rc, pol)[0], q, d, 1e-4)
    # E_real is quadratic in q: the central difference is exact up to rounding
    assert abs(g @ d - fd) <= 1e-9 * np.abs(g).sum()


@pytest.mark.parametrize("which", ["r", "q", "mu", "all"])
def test_real_hvp_finite_difference(which):
    pos, z, box, pol = _sys(n=10, seed=2)
    rng = np.random.default_rng(1)
    n = len(z)
    q = z + 0.2 * rng.normal(size=n)
    mu = 0.3 * rng.normal(size=(n, 3))
    alpha, rc = 0.35, 5.5
    vp = rng.normal(size=(n, 3)) if which in ("r", "all") else np.zeros((n, 3))
    vq = rng.normal(size=n) if which in ("q", "all") else np.zeros(n)
    vm = rng.normal(size=(n, 3)) if which in ("mu", "all") else np.zeros((n, 3))
    h_q, h_mu = opol.real_hvp(pos, q, mu, box, alpha, rc, pol, vp, vq, vm)

    def grads(t):
        P, Q, M = pos + t * vp, q + t * vq, mu + t * vm
        return (opol.real_charge_grad(P, Q, M, box, alpha, rc, pol),
                opol.real_space(P, Q, M, box, alpha, rc, pol)[2])

    hh = 1e-5
    (qp, mp), (qm, mm) = grads(hh), grads(-hh)
    fq, fm = (qp - qm) / (2 * hh), (mp - mm) / (2 * hh)
    assert np.abs(h_q - fq).max() <= 1e-6 * np.abs(fq).max()
    assert np.abs(h_mu - fm).max() <= 1e-6 * np.abs(fm).max()


def test_model_charge_gradient_and_hvp_finite_difference():
    pos, z, box, pol = _sys(n=8, seed=3)
    rng = np.random.default_rng(2)
    n = len(z)
    q = z + 0.2 * rng.normal(size=n)
    mu = 0.3 * rng.normal(size=(n, 3))
    mesh, p, alpha, rc = (10, 10, 10), 5, 0.35, 5.5
    U, Ur, Uq, Umu = opol.model_grads(pos, q, mu, box, mesh, p, alpha, rc, pol)
    d = rng.normal(size=n)
    fd = _cd(lambda qq: opol.model(pos, qq, mu, box, mesh, p, alpha, rc, pol)[0], q, d, 1e-4)
    assert abs(Uq @ d - fd) <= 1e-9 * np.abs(Uq).sum()
    vp, vq, vm = rng.normal(size=(n, 3)), rng.normal(size=n), rng.normal(size=(n, 3))
    h_q, h_mu = opol.model_hvp(pos, q, mu, box, mesh, p, alpha, rc, pol, vp, vq, vm)
    hh = 1e-5
    gp = opol.model_grads(pos + hh * vp, q + hh * vq, mu + hh * vm, box, mesh, p, alpha, rc, pol)
    gm = opol.model_grads(pos - hh * vp, q - hh * vq, mu - hh * vm, box, mesh, p, alpha, rc, pol)
    fq, fm = (gp[2] - gm[2]) / (2 * hh), (gp[3] - gm[3]) / (2 * hh)
    assert np.abs(h_q - fq).max() <= 1e-6 * np.abs(fq).max()
    assert np.abs(h_mu - fm).max() <= 1e-6 * np.abs(fm).max()


def test_feature_tangent_and_transpose():
    pos, z, box, _ = _sys(n=14, seed=5)
    rc = 5.0
    rng = np.random.default_rng(3)
    v = rng.normal(size=pos.shape)
    xd, Vd = oh.features_jvp(pos, z, box, rc, v)
    h = 1e-5
    xp, Vp = odip.features(pos + h * v, z, box, rc)
    xm, Vm = odip.features(pos - h * v, z, box, rc)
    assert np.abs(xd - (xp - xm) / (2 * h)).max() <= 1e-6 * np.abs(xd).max()
    assert np.abs(Vd - (Vp - Vm) / (2 * h)).max() <= 1e-6 * np.abs(Vd).max()
    assert np.all(xd[:, 2 * odip.NCH:] == 0.0)
    gx, gV = rng.normal(size=xd.shape), rng.normal(size=Vd.shape)
    g = oh.features_vjp(pos, z, box, rc, gx, gV)
    lhs = np.sum(gx * xd) + np.sum(gV * Vd)
    assert abs(np.sum(g * v) - lhs) <= 1e-12 * (np.abs(gx * xd).sum() + np.abs(gV * Vd).sum())


def test_charge_head_invariants():
    pos, z, box, _ = _sys(n=16, seed=6)
    _, thq = _params(4)
    x, _ = odip.features(pos, z, box, 5.0)
    q, _ = oh.charges(thq, x, z)
    assert abs(q.sum() - z.sum()) <= 1e-12 * len(z)
    assert np.abs(q - z).max() > 1e-3                   # the head does move the charges
    # translation and the axis permutations of the cubic cell leave charges unchanged
    x2, _ = odip.features((pos + np.array([1.3, -4.1, 7.7])) % 12.0, z, box, 5.0)
    assert np.abs(oh.charges(thq, x2, z)[0] - q).max() <= 1e-12
    x3, _ = odip.features(pos[:, [2, 0, 1]], z, box, 5.0)
    assert np.abs(oh.charges(thq, x3, z)[0] - q).max() <= 1e-12
    # zero output weights: the formal charges exactly
    t0 = thq.copy()
    t0[-64:] = 0.0
    assert np.array_equal(oh.charges(t0, x, z)[0], z)
    # permuting the atoms permutes the charges
    perm = np.random.default_rng(0).permutation(len(z))
    x4, _ = odip.features(pos[perm], z[perm], box, 5.0)
    assert np.abs(oh.charges(thq, x4, z[perm])[0] - q[perm]).max() <= 1e-12


def test_forward_mode_of_both_heads():
    pos, z, box, _ = _sys(n=12, seed=7)
    theta, thq = _params(5)
    x, V = odip.features(pos, z, box, 5.0)
    rng = np.random.default_rng(4)
    xd = rng.normal(size=x.shape)
    xd[:, 2 * odip.NCH:] = 0.0
    Vd = rng.normal(size=V.shape)
    h = 1e-6
    c, cd, _ = oh.charge_jvp(thq, x, xd)
    fd = (oh.charge_jvp(thq, x + h * xd)[0] - oh.charge_jvp(thq, x - h * xd)[0]) / (2 * h)
    assert np.abs(cd - fd).max() <= 1e-7 * np.abs(fd).max()
    mu, mud, _, _, _ = oh.dipoles_jvp(theta, x, V, xd, Vd)
    fd = (odip.dipoles(theta, x + h * xd, V + h * Vd)[0]
          - odip.dipoles(theta, x - h * xd, V - h * Vd)[0]) / (2 * h)
    assert np.abs(mud - fd).max() <= 1e-7 * np.abs(fd).max()


def test_dual_backward_finite_difference():
    pos, z, box, _ = _sys(n=12, seed=8)
    theta, thq = _params(6)
    x, V = odip.features(pos, z, box, 5.0)
    rng = np.random.default_rng(5)
    xd = rng.normal(size=x.shape)
    gc, gcd = rng.normal(size=len(z)), rng.normal(size=len(z))
    gw, gwd = rng.normal(size=(len(z), odip.NCH)), rng.normal(size=(len(z), odip.NCH))

    def fq(t):
        c, cd, _ = oh.charge_jvp(t, x, xd)
        return gc @ c + gcd @ cd

    def fm(t):
        w, wd, _ = oh.mlp_jvp(t, x, xd)
        return np.sum(gw * w) + np.sum(gwd * wd)

    g_q = oh.charge_jvp_backward(thq, oh.charge_jvp(thq, x, xd)[2], gc, gcd)
    g_m = oh.mlp_jvp_backward(theta, oh.mlp_jvp(theta, x, xd)[2], gw, gwd)
    for seed in range(3):
        d = np.random.default_rng(10 + seed)
        dq, dm = d.normal(size=thq.size), d.normal(size=theta.size)
        assert abs(g_q @ dq - _cd(fq, thq, dq, 1e-6)) <= 1e-7 * np.abs(g_q * dq).sum()
        assert abs(g_m @ dm - _cd(fm, theta, dm, 1e-6)) <= 1e-7 * np.abs(g_m * dm).sum()
    # the first-order case agrees with the plain reverse pass of oracle/dip
    _, cache = odip.mlp(theta, x)
    g0 = oh.mlp_jvp_backward(theta, oh.mlp_jvp(theta, x, xd)[2], gw, np.zeros_like(gwd))
    assert np.abs(g0 - odip.mlp_backward(theta, cache, gw)).max() <= 1e-12 * np.abs(g0).max()


def test_head_position_vjp_finite_difference():
    pos, z, box, _ = _sys(n=12, seed=9)
    theta, thq = _params(7)
    rc = 5.0
    rng = np.random.default_rng(6)
    u, c = rng.normal(size=pos.shape), rng.normal(size=len(z))
    g = oh.position_vjp(theta, thq, pos, z, box, rc, u, c)

    def f(P):
        x, V = odip.features(P, z, box, rc)
        return np.sum(u * odip.dipoles(theta, x, V)[0]) + c @ oh.charges(thq, x, z)[0]

    for s in range(4):
        d = np.random.default_rng(20 + s).normal(size=pos.shape)
        fd = _cd(f, pos, d, 1e-5)
        assert abs(np.sum(g * d) - fd) <= 1e-7 * np.abs(g * d).sum()
    assert np.abs(g.sum(axis=0)).max() <= 1e-11 * np.abs(g).max() * len(z)
    # without the charge cotangent it is the dipole-only product of oracle/dip
    g_mu = oh.position_vjp(theta, thq, pos, z, box, rc, u, None)
    assert np.abs(g_mu - odip.position_vjp(theta, pos, z, box, rc, u)).max() <= 1e-12 * np.abs(g_mu).max()


MESH, P, ALPHA, RC = (10, 10, 10), 5, 0.35, 5.5


def _teacher(pos, z, box, pol):
    mu_t = opol.induced_dipoles(pos, z, box, MESH, P, ALPHA, RC, pol)
    U, dUdr, _ = opol.model(pos, z, mu_t, box, MESH, P, ALPHA, RC, pol)
    return {"U": U, "dUdr": dUdr, "mu": mu_t}


def test_conservative_force_with_charge_head():
    pos, z, box, pol = _sys(n=8, seed=10)
    theta, thq = _params(8)
    s = oh.student(theta, thq, pos, z, pol, box, MESH, P, ALPHA, RC)

    def total(Pp):
        x, V = odip.features(Pp, z, box, 5.0)
        q, _ = oh.charges(thq, x, z)
        mu = odip.dipoles(theta, x, V)[0]
        return opol.model(Pp, q, mu, box, MESH, P, ALPHA, RC, pol)[0]

    for s_ in range(3):
        d = np.random.default_rng(30 + s_).normal(size=pos.shape)
        fd = _cd(total, pos, d, 1e-5)
        assert abs(-np.sum(s["F"] * d) - fd) <= 1e-7 * np.abs(s["F"] * d).sum()
    # the charge channel matters: dropping it changes the force
    no_q = s["Ur"] + oh.position_vjp(theta, thq, pos, z, box, 5.0, s["Umu"], None)
    assert np.abs(-s["F"] - no_q).max() > 1e-3 * np.abs(s["F"]).max()


@pytest.mark.parametrize("conservative", [True, False])
def test_loss_gradient_finite_difference(conservative):
    pos, z, box, pol = _sys(n=8, seed=11)
    theta, thq = _params(9)
    # the teacher on a displaced copy, so the loss is far from a minimum
    teacher = _teacher(pos + np.random.default_rng(7).normal(scale=0.05, size=pos.shape),
                       z, box, pol)
    kw = dict(lE=1.0, lF=1.0, lmu=0.5, conservative=conservative)
    args = (pos, z, pol, box, MESH, P, ALPHA, RC, teacher)
    L, g_t, g_q = oh.loss_and_grad(theta, thq, *args, **kw)
    assert L == pytest.approx(oh.loss(theta, thq, *args, **kw), rel=1e-13)
    for s in range(2):
        rng = np.random.default_rng(40 + s)
        dt, dq = rng.normal(size=theta.size), rng.normal(size=thq.size)
        fd_t = _cd(lambda t: oh.loss(t, thq, *args, **kw), theta, dt, 1e-6)
        fd_q = _cd(lambda t: oh.loss(theta, t, *args, **kw), thq, dq, 1e-6)
        assert abs(g_t @ dt - fd_t) <= 1e-6 * np.abs(g_t * dt).sum(), (g_t @ dt, fd_t)
        assert abs(g_q @ dq - fd_q) <= 1e-6 * np.abs(g_q * dq).sum(), (g_q @ dq, fd_q)
