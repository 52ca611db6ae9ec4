"""Pins of the dipole-head oracle (oracle/dip.py), FP64 on the CPU.

* The envelope reaches zero at r_c with zero first and second derivatives. The
  radial functions without it are orthonormal with weight r^2 on [0, r_c].
* Features agree with a plain double loop. They are rotation invariant and
  translation invariant, while the vector channels and dipoles rotate with the
  structure.
* MLP parameter gradients match central differences.
* The training gradient through the PME model matches central differences of the
  loss. This pins the chain through the Hessian-vector product and the mixed
  real-space block.
"""
import math

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


def test_envelope_and_radial_basis():
    assert odip.envelope(0.0) == 1.0
    assert abs(float(odip.envelope(1.0 - 1e-12))) < 1e-9
    h = 1e-4
    f = lambda x: 1 - 21 * x ** 5 + 35 * x ** 6 - 15 * x ** 7
    assert abs((f(1 + h) - f(1 - h)) / (2 * h)) < 1e-6
    assert abs((f(1 + h) - 2 * f(1) + f(1 - h)) / h ** 2) < 1e-4
    rc = 5.0
    r = np.linspace(1e-6, rc, 200001)
    k = np.arange(1, odip.NRAD + 1)
    B = math.sqrt(2 / rc) * np.sin(np.outer(r, k) * math.pi / rc) / r[:, None]
    gram = np.trapezoid(B[:, :, None] * B[:, None, :] * (r ** 2)[:, None, None], r, axis=0)
    np.testing.assert_allclose(gram, np.eye(odip.NRAD), atol=1e-6)


def test_features_match_double_loop():
    pos, q, box, _ = _sys(n=8)
    rc = 5.0
    x, V = odip.features(pos, q, box, rc)
    L = box[0, 0]
    G2 = np.zeros((8, 2, 8))
    V2 = np.zeros((8, 2, 8, 3))
    for i in range(8):
        for j in range(8):
            for a in range(-1, 2):
                for b in range(-1, 2):
                    for c in range(-1, 2):
                        R = pos[i] - pos[j] + L * np.array([a, b, c])
                        r = np.linalg.norm(R)
                        if r < 1e-12 or r >= rc:
                            continue
                        s = 0 if q[j] > 0 else 1
                        for k in range(8):
                            val = math.sqrt(2 / rc) * math.sin((k + 1) * math.pi * r / rc) / r
                            val *= float(odip.envelope(r / rc))
                            G2[i, s, k] += val
                            V2[i, s, k] += q[j] * val * R / r
    np.testing.assert_allclose(x[:, :16], G2.reshape(8, 16), atol=1e-12)
    np.testing.assert_allclose(V, V2.reshape(8, 16, 3), atol=1e-12)
    np.testing.assert_allclose(x[:, 16:32], (V2.reshape(8, 16, 3) ** 2).sum(-1), atol=1e-12)


def test_rotation_and_translation():
    pos, q, box, _ = _sys(n=10, seed=5)
    theta = synth.mlp_init(3, last_scale=1.0)
    x, V = odip.features(pos, q, box, 5.0)
    mu, _, _ = odip.dipoles(theta, x, V)
    # rotate the whole periodic system (cell rows and positions)
    ang = 0.7
    Rm = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    Rm = Rm @ np.array([[1, 0, 0], [0, math.cos(0.3), -math.sin(0.3)], [0, math.sin(0.3), math.cos(0.3)]])
    x2, V2 = odip.features(pos @ Rm.T, q, box @ Rm.T, 5.0)
    np.testing.assert_allclose(x2, x, atol=1e-10)
    mu2, _, _ = odip.dipoles(theta, x2, V2)
    np.testing.assert_allclose(mu2, mu @ Rm.T, atol=1e-10)
    x3, V3 = odip.features(pos + np.array([1.3, -2.2, 0.4]), q, box, 5.0)
    np.testing.assert_allclose(x3, x, atol=1e-10)
    np.testing.assert_allclose(V3, V, atol=1e-10)


def test_mlp_backward_finite_difference():
    rng = np.random.default_rng(0)
    theta = synth.mlp_init(1, last_scale=1.0)
    x = rng.normal(0, 1, (5, odip.NFEAT))
    gw = rng.normal(0, 1, (5, odip.NCH))
    w, cache = odip.mlp(theta, x)
    g = odip.mlp_backward(theta, cache, gw)
    h = 1e-6
    for k in rng.choice(odip.NPARAM, 12, replace=False):
        d = np.zeros(odip.NPARAM)
        d[k] = h
        fp = float(np.sum(odip.mlp(theta + d, x)[0] * gw))
        fm = float(np.sum(odip.mlp(theta - d, x)[0] * gw))
        assert abs((fp - fm) / (2 * h) - g[k]) < 1e-7 * (1 + abs(g[k]))


@pytest.mark.slow
def test_training_gradient_through_pme_finite_difference():
    pos, q, box, pol = _sys(n=8, seed=6)
    mesh, p, alpha, rc = (12, 12, 12), 5, 0.35, 5.5
    mu_t = opol.induced_dipoles(pos, q, box, mesh, p, alpha, rc, pol)
    U, dUdr, _ = opol.model(pos, q, mu_t, box, mesh, p, alpha, rc, pol)
    teacher = {"U": U, "dUdr": dUdr, "mu": mu_t}
    theta = synth.mlp_init(2, last_scale=1.0)
    x, V = odip.features(pos, q, box, 5.0)
    L, g, _ = odip.loss_and_grad(theta, x, V, pos, q, pol, box, mesh, p, alpha, rc, teacher,
                                 lE=1.0, lF=1.0, lmu=0.5)
    h = 1e-6
    rng = np.random.default_rng(1)
    for k in list(rng.choice(odip.NPARAM, 6, replace=False)) + [odip.NPARAM - 1]:
        d = np.zeros(odip.NPARAM)
        d[k] = h
        Lp = odip.loss_and_grad(theta + d, x, V, pos, q, pol, box, mesh, p, alpha, rc, teacher,
                                1.0, 1.0, 0.5)[0]
        Lm = odip.loss_and_grad(theta - d, x, V, pos, q, pol, box, mesh, p, alpha, rc, teacher,
                                1.0, 1.0, 0.5)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * (abs(g).max()), (k, fd, g[k])
