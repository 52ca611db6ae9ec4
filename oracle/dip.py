"""Learned dipole head on local features, trained through PME (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

This follows the dipole readout of Sec. 2.2 (Eq. dipole_pred): a dipole is an
invariant-weighted sum of equivariant vector features of the atom's
neighbourhood. The paper's HotPP backbone is replaced by fixed features within
r_c = 5 A:

    radial   R_k(r) = sqrt(2 / r_c) sin(k pi r / r_c) / r * f(r / r_c),  k = 1..8
    envelope f(x)   = 1 - 21 x^5 + 35 x^6 - 15 x^7 (x < 1; 0 beyond), the
                      polynomial envelope of order 5
    scalars  G_i[s, k] = sum_{j of species s} R_k(r_ij)
    vectors  V_i[s, k] = sum_{j of species s} q_j R_k(r_ij) R_ij / r_ij,
             R_ij = r_i - r_j (minimum image)
    inputs   x_i = [G_i (16), |V_i[c]|^2 (16), one-hot species of i (2)]   (34)

The species are cation (q > 0) and anion.

An MLP with two SiLU hidden layers of width 64 maps x_i to 16 channel weights w_i, and mu_i = sum_c w_ic V_i[c]. This is rotation covariant and translation invariant.

Flat parameter layout: W1 [64][34], b1 [64], W2 [64][64], b2 [64], W3 [16][64], b3 [16] (7440 values).

Training (Eq. loss, with the teacher of oracle/pol):

    L = l_E ((U_s - U_t) / n)^2 + l_F mean_{i,a} (F_s - F_t)^2 + l_mu mean (mu - mu_t)^2

Here F_s = -dU/dr at mu = mu_NN, the student's Hellmann-Feynman force.

    dL/dmu = (dL/dU_s) dU/dmu + H_{mu r} v,  v = dL/d(dU/dr)

H_{mu r} v is the PME Hessian-vector product (dipole block) plus the real-space mixed block. The gradient then flows through w to the parameters (first order; the features do not depend on them).

Conservative student forces (position_vjp, conservative_forces): F = -dU(r, mu_NN(r))/dr adds to the Hellmann-Feynman force the path through the dipole head, (d mu_NN / dr)^T dU/dmu, which runs back through the network's input gradient and the position derivatives of the features.
"""
from __future__ import annotations

import math

import numpy as np

from . import pme as opme
from . import pol as opol

NRAD = 8
NSPEC = 2
NCH = NRAD * NSPEC
NFEAT = 2 * NCH + NSPEC
HID = 64
SHAPES = [(HID, NFEAT), (HID,), (HID, HID), (HID,), (NCH, HID), (NCH,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta):
    out, k = [], 0
    for s in SHAPES:
        m = int(np.prod(s))
        out.append(np.asarray(theta[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def envelope(x):
    x = np.asarray(x, dtype=np.float64)
    f = 1.0 - 21.0 * x ** 5 + 35.0 * x ** 6 - 15.0 * x ** 7
    return np.where(x < 1.0, f, 0.0)


def radial(r, rc):
    """(len(r), NRAD) radial basis with the envelope."""
    r = np.asarray(r, dtype=np.float64)
    k = np.arange(1, NRAD + 1)
    return (math.sqrt(2.0 / rc) * np.sin(np.outer(r, k) * math.pi / rc) / r[:, None]
            * envelope(r / rc)[:, None])


def features(pos, q, box, rc):
    """Inputs x (n, 34) and vector channels V (n, 16, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    n = pos.shape[0]
    ia, ja, R, r = opol._pairs(pos, box, rc)
    Rk = radial(r, rc)                                    # (P, 8)
    spec = (q[ja] <= 0).astype(int)                       # species of the neighbour
    G = np.zeros((n, NSPEC, NRAD))
    V = np.zeros((n, NSPEC, NRAD, 3))
    np.add.at(G, (ia, spec), Rk)
    np.add.at(V, (ia, spec), (q[ja][:, None] * Rk)[:, :, None] * (R / r[:, None])[:, None, :])
    G = G.reshape(n, NCH)
    V = V.reshape(n, NCH, 3)
    onehot = np.stack([(q > 0).astype(float), (q <= 0).astype(float)], axis=1)
    x = np.concatenate([G, np.einsum('ncd,ncd->nc', V, V), onehot], axis=1)
    return x, V


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mlp(theta, x):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    w = h2 @ W3.T + b3
    return w, (x, z1, h1, z2, h2)


def mlp_backward(theta, cache, gw):
    """Parameter gradient (flat) from dL/dw (n, 16)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    x, z1, h1, z2, h2 = cache
    gW3 = gw.T @ h2
    gb3 = gw.sum(0)
    gz2 = (gw @ W3) * dsilu(z2)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(0)
    gz1 = (gz2 @ W2) * dsilu(z1)
    gW1 = gz1.T @ x
    gb1 = gz1.sum(0)
    return np.concatenate([a.reshape(-1) for a in (gW1, gb1, gW2, gb2, gW3, gb3)])


def dipoles(theta, x, V):
    w, cache = mlp(theta, x)
    return np.einsum('nc,ncd->nd', w, V), w, cache


def radial_derivative(r, rc):
    """(len(r), NRAD) derivative of the radial basis with respect to r."""
    r = np.asarray(r, dtype=np.float64)
    k = np.arange(1, NRAD + 1)
    x = r / rc
    env = envelope(x)[:, None]
    denv = (np.where(x < 1.0, -105.0 * x ** 4 + 210.0 * x ** 5 - 105.0 * x ** 6, 0.0) / rc)[:, None]
    arg = np.outer(r, k) * math.pi / rc
    sn, cs = np.sin(arg), np.cos(arg)
    rr = r[:, None]
    return math.sqrt(2.0 / rc) * ((k * math.pi / rc) * cs / rr * env - sn / rr ** 2 * env
                                  + sn / rr * denv)


def mlp_input_grad(theta, cache, gw):
    """dL/dx (n, 34) from dL/dw (n, 16): the network's input gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    x, z1, h1, z2, h2 = cache
    gz2 = (gw @ W3) * dsilu(z2)
    gz1 = (gz2 @ W2) * dsilu(z1)
    return gz1 @ W1


def position_vjp(theta, pos, q, box, rc, u):
    """g_j = sum_i (d mu_i / d r_j)^T u_i: the total derivative of the dipole head with
    respect to the positions, contracted with u (n, 3).

    mu_i depends on the positions through its features (the charges and species are
    fixed): with cotangents cG = dL/dG_i and cV = dL/dV_i (from w_ic u_i and the
    input gradient of |V_ic|^2), a pair R = r_i - r_j with neighbour j of species s
    contributes, per radial k,
        d/dR [cG R_k(r)]              = cG R_k'(r) u_hat
        d/dR [q_j R_k(r) cV . u_hat]  = q_j [R_k'(r) (cV . u_hat) u_hat
                                            + R_k(r)/r (cV - (cV . u_hat) u_hat)]
    to r_i and the negative to r_j."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = pos.shape[0]
    x, V = features(pos, q, box, rc)
    _, w, cache = dipoles(theta, x, V)
    gw = np.einsum('nd,ncd->nc', u, V)
    gx = mlp_input_grad(theta, cache, gw)
    cG = gx[:, :NCH].reshape(n, NSPEC, NRAD)
    cV = (w[:, :, None] * u[:, None, :] + 2.0 * gx[:, NCH:2 * NCH, None] * V).reshape(
        n, NSPEC, NRAD, 3)
    ia, ja, R, r = opol._pairs(pos, box, rc)
    Rk = radial(r, rc)
    dRk = radial_derivative(r, rc)
    uh = R / r[:, None]
    spec = (q[ja] <= 0).astype(int)
    cg = cG[ia, spec]                                  # (P, 8)
    cv = cV[ia, spec]                                  # (P, 8, 3)
    cu = np.einsum('pkd,pd->pk', cv, uh)
    f = (np.einsum('pk,pk->p', cg, dRk)[:, None] * uh
         + q[ja][:, None] * (np.einsum('pk,pk->p', cu, dRk)[:, None] * uh
                             + np.einsum('pk,pkd->pd', Rk / r[:, None],
                                         cv - cu[:, :, None] * uh[:, None, :])))
    g = np.zeros((n, 3))
    np.add.at(g, ia, f)
    np.add.at(g, ja, -f)
    return g


def conservative_forces(theta, pos, q, pol, box, mesh, p, alpha, rc, rc_feat=5.0):
    """Student forces as the total derivative F = -dU(r, mu_NN(r))/dr (the conservative
    alternative to the Hellmann-Feynman force of Eq. loss), the energy and the dipoles;
    rc is the real-space cutoff of the model, rc_feat that of the features."""
    x, V = features(pos, q, box, rc_feat)
    mu, _, _ = dipoles(theta, x, V)
    U, dUdr, dUdmu = opol.model(pos, q, mu, box, mesh, p, alpha, rc, pol)
    return -(dUdr + position_vjp(theta, pos, q, box, rc_feat, dUdmu)), U, mu


def loss_and_grad(theta, x, V, pos, q, pol, box, mesh, p, alpha, rc, teacher, lE=1.0, lF=1.0,
                  lmu=0.0):
    """L and dL/dtheta through the model (teacher: dict U, dUdr, mu)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    mu, w, cache = dipoles(theta, x, V)
    U, dUdr, dUdmu = opol.model(pos, q, mu, box, mesh, p, alpha, rc, pol)
    dE = (U - teacher["U"]) / n
    dF = dUdr - teacher["dUdr"]                      # = -(F_s - F_t)
    dM = mu - teacher["mu"]
    L = lE * dE * dE + lF * float(np.mean(dF * dF)) + lmu * float(np.mean(dM * dM))
    cE = 2.0 * lE * dE / n                           # dL/dU
    v = 2.0 * lF * dF / dF.size                      # dL/d(dU/dr)
    _, _, h_pme = opme.hvp(pos, q, mu, box, mesh, p, alpha, v, None, None)
    h_real = opol.real_mixed(pos, q, mu, box, alpha, rc, pol, v)
    g_mu = cE * dUdmu + h_pme + h_real + 2.0 * lmu * dM / dM.size
    gw = np.einsum('nd,ncd->nc', g_mu, V)
    return L, mlp_backward(theta, cache, gw), mu
