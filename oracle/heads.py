"""Charge head and training on conservative forces (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Charge head (Sec. 2.2, Eq. charge_pred).  A two-layer perceptron with SiLU maps
the scalar inputs x_i of oracle/dip.features (34 invariants) to

    c_i = w2 . silu(W1 x_i + b1),        W1 [64][34], b1 [64], w2 [64] (2304 values)

and the charges are the formal charges z_i plus these contributions with their
mean removed,

    q_i = z_i + c_i - (1/n) sum_k c_k,

so the cell keeps the total charge sum z (the PME energy leaves out k = 0, which
assumes a neutral cell).  An output bias would cancel in the centring and is
left out.  The features themselves (species, the charge weights of the vector
channels) use the formal charges z, so they do not depend on the parameters.

Student model.  U(r) = U_pol(r, q(r), mu(r)) with U_pol the polarizable model of
oracle/pol (E_lr + E_real + polarization), q the charge head and mu the dipole
head of oracle/dip.

Conservative forces (Eq. forces).  F = -dU/dr with every channel:

    dU/dr = U_r + J_q^T U_q + J_mu^T U_mu,

U_r, U_q, U_mu the partial gradients of U_pol and J the head Jacobians in r.

Training on them (Eq. loss).

    L = lE ((U_s - U_t)/n)^2 + lF mean (F_s - F_t)^2 + lmu mean (mu - mu_t)^2

With a = dL/dU and v = dL/d(dU/dr), the force term is Phi(theta) = v . dU/dr, the
derivative of U along the positions in direction v.  Derivatives in theta and
along v commute, so

    dPhi/dtheta = (H_q. t)^T dq/dtheta + (H_mu. t)^T dmu/dtheta
                  + U_q^T d(q_dot)/dtheta + U_mu^T d(mu_dot)/dtheta,

where t = (v, q_dot, mu_dot) is the full tangent (q_dot = J_q v, mu_dot = J_mu v),
H_q. t and H_mu. t are the q and mu rows of the Hessian of U_pol applied to t
(oracle/pol.model_hvp), and q_dot, mu_dot are the heads' forward-mode
derivatives along the feature tangent x_dot = J_x v, which does not depend on
the parameters.  The parameter gradient is therefore reverse mode through the
heads' forward-mode (dual) evaluation with cotangents

    on q:      a U_q + H_q. t        on q_dot:   U_q
    on mu:     a U_mu + H_mu. t      on mu_dot:  U_mu

(the centring maps a charge cotangent g to g - mean g).  The Hellmann-Feynman
alternative F = -U_r keeps only t = (v, 0, 0) and no q_dot, mu_dot cotangents.
"""
from __future__ import annotations

import numpy as np

from . import dip as odip
from . import pme as opme
from . import pol as opol

HID = odip.HID
NFEAT = odip.NFEAT
NCH = odip.NCH
NRAD = odip.NRAD
NSPEC = odip.NSPEC
QSHAPES = [(HID, NFEAT), (HID,), (HID,)]
NQPARAM = sum(int(np.prod(s)) for s in QSHAPES)


def unpack_q(thq):
    out, k = [], 0
    for s in QSHAPES:
        m = int(np.prod(s))
        out.append(np.asarray(thq[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def d2silu(z):
    """Second derivative of z sigma(z): sigma (1 - sigma) (2 + z (1 - 2 sigma))."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def centre(a):
    return a - a.mean(axis=0)


# ---- charge head ----

def charge_jvp(thq, x, xd=None):
    """c (n,) and its directional derivative c_dot along the input tangent xd."""
    W1, b1, w2 = unpack_q(thq)
    xd = np.zeros_like(x) if xd is None else xd
    z = x @ W1.T + b1
    zd = xd @ W1.T
    h = odip.silu(z)
    hd = odip.dsilu(z) * zd
    return h @ w2, hd @ w2, (x, xd, z, zd, h, hd)


def charges(thq, x, z_formal, xd=None):
    """q = z + centred c, and q_dot = centred c_dot (Eq. charge_pred with neutrality)."""
    c, cd, _ = charge_jvp(thq, x, xd)
    return np.asarray(z_formal, dtype=np.float64) + centre(c), centre(cd)


def charge_input_grad(thq, x, gc):
    """dL/dx (n, 34) from a cotangent gc on c."""
    W1, b1, w2 = unpack_q(thq)
    z = x @ W1.T + b1
    return ((gc[:, None] * w2[None, :]) * odip.dsilu(z)) @ W1


def charge_jvp_backward(thq, cache, gc, gcd):
    """Parameter gradient from cotangents gc on c and gcd on c_dot."""
    W1, b1, w2 = unpack_q(thq)
    x, xd, z, zd, h, hd = cache
    gw2 = gc @ h + gcd @ hd
    gh = gc[:, None] * w2[None, :]
    ghd = gcd[:, None] * w2[None, :]
    gz = gh * odip.dsilu(z) + ghd * d2silu(z) * zd
    gzd = ghd * odip.dsilu(z)
    gW1 = gz.T @ x + gzd.T @ xd
    return np.concatenate([gW1.reshape(-1), gz.sum(0), gw2])


# ---- dipole head in forward mode ----

def mlp_jvp(theta, x, xd):
    """The dipole network's outputs w and their directional derivatives wd."""
    W1, b1, W2, b2, W3, b3 = odip.unpack(theta)
    z1 = x @ W1.T + b1
    z1d = xd @ W1.T
    h1, h1d = odip.silu(z1), odip.dsilu(z1) * z1d
    z2 = h1 @ W2.T + b2
    z2d = h1d @ W2.T
    h2, h2d = odip.silu(z2), odip.dsilu(z2) * z2d
    return h2 @ W3.T + b3, h2d @ W3.T, (x, xd, z1, z1d, h1, h1d, z2, z2d, h2, h2d)


def mlp_jvp_backward(theta, cache, gw, gwd):
    """Parameter gradient (flat) from cotangents gw on w and gwd on wd."""
    W1, b1, W2, b2, W3, b3 = odip.unpack(theta)
    x, xd, z1, z1d, h1, h1d, z2, z2d, h2, h2d = cache
    gW3 = gw.T @ h2 + gwd.T @ h2d
    gb3 = gw.sum(0)
    gh2, gh2d = gw @ W3, gwd @ W3
    gz2 = gh2 * odip.dsilu(z2) + gh2d * d2silu(z2) * z2d
    gz2d = gh2d * odip.dsilu(z2)
    gW2 = gz2.T @ h1 + gz2d.T @ h1d
    gb2 = gz2.sum(0)
    gh1, gh1d = gz2 @ W2, gz2d @ W2
    gz1 = gh1 * odip.dsilu(z1) + gh1d * d2silu(z1) * z1d
    gz1d = gh1d * odip.dsilu(z1)
    gW1 = gz1.T @ x + gz1d.T @ xd
    gb1 = gz1.sum(0)
    return np.concatenate([a.reshape(-1) for a in (gW1, gb1, gW2, gb2, gW3, gb3)])


def dipoles_jvp(theta, x, V, xd, Vd):
    """mu and mu_dot = sum_c (wd_c V_c + w_c Vd_c)."""
    w, wd, cache = mlp_jvp(theta, x, xd)
    mu = np.einsum('nc,ncd->nd', w, V)
    mud = np.einsum('nc,ncd->nd', wd, V) + np.einsum('nc,ncd->nd', w, Vd)
    return mu, mud, w, wd, cache


# ---- features: tangent and transpose ----

def _pair_terms(pos, z_formal, box, rc):
    z_formal = np.asarray(z_formal, dtype=np.float64)
    ia, ja, R, r = opol._pairs(np.asarray(pos, dtype=np.float64), box, rc)
    spec = (z_formal[ja] <= 0).astype(int)
    return ia, ja, R, r, R / r[:, None], spec, odip.radial(r, rc), odip.radial_derivative(r, rc)


def features_jvp(pos, z_formal, box, rc, v):
    """Directional derivatives of oracle/dip.features along positions v (n, 3):
    x_dot (n, 34) and V_dot (n, 16, 3).  For a pair R = r_i - r_j, w = v_i - v_j,
    u = R/r and r_dot = u . w:
        G_dot[s, k] += R_k'(r) r_dot
        V_dot[s, k] += z_j [R_k'(r) r_dot u + R_k(r)/r (w - r_dot u)]
    and the tangent of |V_c|^2 is 2 V_c . V_dot_c; the one-hot entries are fixed."""
    pos = np.asarray(pos, dtype=np.float64)
    z_formal = np.asarray(z_formal, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    n = pos.shape[0]
    ia, ja, R, r, u, spec, Rk, dRk = _pair_terms(pos, z_formal, box, rc)
    w = v[ia] - v[ja]
    rd = np.einsum('pc,pc->p', u, w)
    Gd = np.zeros((n, NSPEC, NRAD))
    Vd = np.zeros((n, NSPEC, NRAD, 3))
    np.add.at(Gd, (ia, spec), dRk * rd[:, None])
    perp = w - rd[:, None] * u
    contrib = z_formal[ja][:, None, None] * (
        (dRk * rd[:, None])[:, :, None] * u[:, None, :]
        + (Rk / r[:, None])[:, :, None] * perp[:, None, :])
    np.add.at(Vd, (ia, spec), contrib)
    Gd = Gd.reshape(n, NCH)
    Vd = Vd.reshape(n, NCH, 3)
    _, V = odip.features(pos, z_formal, box, rc)
    xd = np.concatenate([Gd, 2.0 * np.einsum('ncd,ncd->nc', V, Vd), np.zeros((n, NSPEC))], axis=1)
    return xd, Vd


def features_vjp(pos, z_formal, box, rc, gx, gV):
    """Transpose of features_jvp: sum over features of gx . x_dot + gV . V_dot as a
    gradient in the positions (n, 3), for cotangents gx (n, 34) and gV (n, 16, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    z_formal = np.asarray(z_formal, dtype=np.float64)
    n = pos.shape[0]
    _, V = odip.features(pos, z_formal, box, rc)
    cG = gx[:, :NCH].reshape(n, NSPEC, NRAD)
    cV = (gV + 2.0 * gx[:, NCH:2 * NCH, None] * V).reshape(n, NSPEC, NRAD, 3)
    ia, ja, R, r, u, spec, Rk, dRk = _pair_terms(pos, z_formal, box, rc)
    cg = cG[ia, spec]
    cv = cV[ia, spec]
    # d x_dot / d w for one pair, transposed: G part gives cg.dRk u; V part gives
    # z_j [dRk (cv.u) u + Rk/r (cv - (cv.u) u)] summed over k
    cu = np.einsum('pkd,pd->pk', cv, u)
    f = (np.einsum('pk,pk->p', cg, dRk)[:, None] * u
         + z_formal[ja][:, None] * (np.einsum('pk,pk->p', cu, dRk)[:, None] * u
                                    + np.einsum('pk,pkd->pd', Rk / r[:, None],
                                                cv - cu[:, :, None] * u[:, None, :])))
    g = np.zeros((n, 3))
    np.add.at(g, ia, f)
    np.add.at(g, ja, -f)
    return g


def position_vjp(theta, thq, pos, z_formal, box, rc, u=None, c=None):
    """sum_i (d mu_i/dr)^T u_i + (d q_i/dr)^T c_i as a gradient in the positions:
    the head channels of Eq. forces for cotangents u (n, 3) on the dipoles and c
    (n,) on the charges (either may be None)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    x, V = odip.features(pos, z_formal, box, rc)
    gx = np.zeros((n, NFEAT))
    gV = np.zeros((n, NCH, 3))
    if u is not None:
        u = np.asarray(u, dtype=np.float64)
        w, cache = odip.mlp(theta, x)
        gx += odip.mlp_input_grad(theta, cache, np.einsum('nd,ncd->nc', u, V))
        gV += w[:, :, None] * u[:, None, :]
    if c is not None:
        gx += charge_input_grad(thq, x, centre(np.asarray(c, dtype=np.float64)))
    return features_vjp(pos, z_formal, box, rc, gx, gV)


# ---- student model and its training gradient ----

def student(theta, thq, pos, z_formal, pol, box, mesh, p, alpha, rc, rc_feat=5.0,
            conservative=True):
    """Energy, forces, charges and dipoles of the student; the forces are the
    conservative -dU/dr (or the Hellmann-Feynman -U_r)."""
    x, V = odip.features(pos, z_formal, box, rc_feat)
    q, _ = charges(thq, x, z_formal)
    mu, _, _ = odip.dipoles(theta, x, V)
    U, Ur, Uq, Umu = opol.model_grads(pos, q, mu, box, mesh, p, alpha, rc, pol)
    G = Ur + (position_vjp(theta, thq, pos, z_formal, box, rc_feat, Umu, Uq) if conservative
              else 0.0)
    return {"U": U, "F": -G, "q": q, "mu": mu, "Ur": Ur, "Uq": Uq, "Umu": Umu}


def loss(theta, thq, pos, z_formal, pol, box, mesh, p, alpha, rc, teacher, lE=1.0, lF=1.0,
         lmu=0.0, rc_feat=5.0, conservative=True):
    n = len(z_formal)
    s = student(theta, thq, pos, z_formal, pol, box, mesh, p, alpha, rc, rc_feat, conservative)
    dE = (s["U"] - teacher["U"]) / n
    dF = s["F"] + teacher["dUdr"]                 # F_s - F_t, teacher forces -dUdr_t
    L = lE * dE * dE + lF * float(np.mean(dF * dF))
    if lmu:
        dM = s["mu"] - teacher["mu"]
        L += lmu * float(np.mean(dM * dM))
    return L


def loss_and_grad(theta, thq, pos, z_formal, pol, box, mesh, p, alpha, rc, teacher, lE=1.0,
                  lF=1.0, lmu=0.0, rc_feat=5.0, conservative=True):
    """L and (dL/dtheta, dL/dthq) of the student against the teacher (dict U, dUdr,
    and mu when lmu > 0), by the dual-mode rule of the module header."""
    pos = np.asarray(pos, dtype=np.float64)
    z_formal = np.asarray(z_formal, dtype=np.float64)
    n = pos.shape[0]
    x, V = odip.features(pos, z_formal, box, rc_feat)
    q, _ = charges(thq, x, z_formal)
    mu, _, _ = odip.dipoles(theta, x, V)
    U, Ur, Uq, Umu = opol.model_grads(pos, q, mu, box, mesh, p, alpha, rc, pol)
    if conservative:
        G = Ur + position_vjp(theta, thq, pos, z_formal, box, rc_feat, Umu, Uq)
    else:
        G = Ur
    dE = (U - teacher["U"]) / n
    dG = G - teacher["dUdr"]                          # = -(F_s - F_t)
    L = lE * dE * dE + lF * float(np.mean(dG * dG))
    a = 2.0 * lE * dE / n                             # dL/dU
    v = 2.0 * lF * dG / dG.size                       # dL/d(dU/dr)
    g_mu = a * Umu
    if lmu:
        dM = mu - teacher["mu"]
        L += lmu * float(np.mean(dM * dM))
        g_mu = g_mu + 2.0 * lmu * dM / dM.size
    if conservative:
        xd, Vd = features_jvp(pos, z_formal, box, rc_feat, v)
        _, qd = charges(thq, x, z_formal, xd)
        _, mud, w, wd, mcache = dipoles_jvp(theta, x, V, xd, Vd)
    else:
        xd, Vd = np.zeros_like(x), np.zeros_like(V)
        qd, mud = np.zeros(n), np.zeros((n, 3))
        w, wd, mcache = mlp_jvp(theta, x, xd)
    h_q, h_mu = opol.model_hvp(pos, q, mu, box, mesh, p, alpha, rc, pol, v, qd, mud)
    gq = a * Uq + h_q
    gmu = g_mu + h_mu
    uq = Uq if conservative else np.zeros(n)
    umu = Umu if conservative else np.zeros((n, 3))
    # dipole head: mu = sum_c w_c V_c, mu_dot = sum_c (wd_c V_c + w_c Vd_c)
    gw = np.einsum('nd,ncd->nc', gmu, V) + np.einsum('nd,ncd->nc', umu, Vd)
    gwd = np.einsum('nd,ncd->nc', umu, V)
    g_theta = mlp_jvp_backward(theta, mcache, gw, gwd)
    _, _, qcache = charge_jvp(thq, x, xd)
    g_thq = charge_jvp_backward(thq, qcache, centre(gq), centre(uq))
    return L, g_theta, g_thq
