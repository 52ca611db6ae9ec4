"""CPU particle-mesh Ewald for charges and dipoles on a given mesh (FP64).

Follows Secs. 2.3.1-2.3.5 of the paper step by step:

1. cell, inverse cell, volume and reciprocal basis            (Sec. 2.3.1)
2. mesh dimensions from a target spacing and strategy          (Eq. mesh_target)
3. fractional and mesh coordinates, stencil, weights           (Sec. 2.3.2, Eq. w3d)
4. charge + dipole effective density on the mesh               (Eq. charge_dipole_assign)
5. full complex DFT of the density                             (Eq. fft)
6. Green's function times the sinc deconvolution factor        (Eqs. Bk, influence, green)
7. potential by the unnormalised inverse DFT (real part)       (Eqs. potential_k, ifft)
8. energy (1/2V) sum rho*phi, self terms                       (Eqs. energy_recip, self_q,
                                                                self_mu, E_lr_total)
9. analytic gradients of E^lr with respect to r, q and mu, and
   the Hessian-vector product of E^lr (what autograd of the
   pipeline yields, Sec. 2.3.5 and Eq. forces)
10. the gradient of E^lr with respect to the cell at fixed Cartesian
   inputs (the stress/virial loss of Sec. 2.4)

Readings of the text (where it is silent or ambiguous):

* the inverse transform is unnormalised, so E_recip = (1/2V) sum_k g |rho~|^2,
  the only normalisation that agrees with the explicit Ewald sum;
* frequency indices are signed (numpy.fft.fftfreq order: Nyquist at -N/2);
* the potential is the real part of the inverse transform (real-to-complex
  semantics), which makes the mesh operator real-symmetric;
* W^(p) is the centered cardinal B-spline M_p, weight on mesh point m is
  M_p(x - m) for the p nearest mesh points; round() for odd p is floor(x+1/2);
* no neutralising-background term: the k = 0 term is dropped, as stated;
* the dipole contributes +mu . grad_r W (bound charge of a point dipole).

Energies are in units of e^2/Angstrom times ``prefactor``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .bspline import bspline

_CHUNK = 32768


# ----------------------------------------------------------------------------
# 1-2. cell and mesh (Sec. 2.3.1)
# ----------------------------------------------------------------------------

def cell(box):
    """C (rows a_x, a_y, a_z), C^-1, V = |det C| and reciprocal rows b = 2 pi C^-T."""
    C = np.asarray(box, dtype=np.float64).reshape(3, 3)
    Cinv = np.linalg.inv(C)
    V = abs(np.linalg.det(C))
    recip = 2.0 * math.pi * Cinv.T
    return C, Cinv, V, recip


def _five_smooth(m: int) -> bool:
    for f in (2, 3, 5):
        while m % f == 0:
            m //= f
    return m == 1


def mesh_dims(box, spacing: float, strategy: str = "smooth"):
    """Eq. mesh_target followed by one of the three mapping strategies."""
    C = np.asarray(box, dtype=np.float64).reshape(3, 3)
    out = []
    for a in C:
        target = math.ceil(2.0 * np.linalg.norm(a) / spacing + 1.0)
        if strategy == "pow2":
            n = 1 << max(0, math.ceil(math.log2(target)))
        elif strategy == "smooth":
            n = target
            while not _five_smooth(n):
                n += 1
        elif strategy == "ceil":
            n = target
        else:
            raise ValueError(strategy)
        out.append(int(n))
    return tuple(out)


# ----------------------------------------------------------------------------
# 3. stencil and weights (Sec. 2.3.2)
# ----------------------------------------------------------------------------

def mesh_coordinates(pos, box, mesh):
    """x_i = (N_x s_x, N_y s_y, N_z s_z) with s = r C^-1 wrapped into [0, 1)."""
    _, Cinv, _, _ = cell(box)
    s = np.asarray(pos, dtype=np.float64) @ Cinv
    s = s - np.floor(s)
    return s * np.asarray(mesh, dtype=np.float64)


def stencil(pos, box, mesh, p: int):
    """Per atom and axis: wrapped mesh indices (N,3,p) and arguments t = x - m (N,3,p).

    Odd p: n = round(x), xi = x - n, stencil offsets u = -(p-1)/2 .. (p-1)/2,
    weight argument xi - u.  Even p: n = floor(x), xi = x - (n + 1/2), the p
    mesh points n-p/2+1 .. n+p/2, weight argument x - m = xi + 1/2 - u.
    """
    x = mesh_coordinates(pos, box, mesh)
    N = np.asarray(mesh, dtype=np.int64)
    if p % 2 == 1:
        n = np.floor(x + 0.5)
        u = np.arange(-(p - 1) // 2, (p - 1) // 2 + 1, dtype=np.float64)
        xi = x - n
        t = xi[..., None] - u
    else:
        n = np.floor(x)
        u = np.arange(-p // 2 + 1, p // 2 + 1, dtype=np.float64)
        xi = x - (n + 0.5)
        t = xi[..., None] + 0.5 - u
    m = n[..., None].astype(np.int64) + u.astype(np.int64)
    idx = np.mod(m, N[None, :, None])
    return idx, t


def jacobian(box, mesh):
    """J[a, b] = d x_a / d r_b = N_a (C^-1)[b, a]."""
    _, Cinv, _, _ = cell(box)
    return np.asarray(mesh, dtype=np.float64)[:, None] * Cinv.T


def _flat(idx, mesh):
    """Flat row-major (z fastest) mesh index for every stencil point: (N, p, p, p)."""
    Nx, Ny, Nz = mesh
    ix, iy, iz = idx[:, 0], idx[:, 1], idx[:, 2]
    return (ix[:, :, None, None] * Ny + iy[:, None, :, None]) * Nz + iz[:, None, None, :]


def _w3(wx, wy, wz, a, b, c):
    """Separable product W_x^(a) W_y^(b) W_z^(c) over the stencil: (N, p, p, p)."""
    return wx[a][:, :, None, None] * wy[b][:, None, :, None] * wz[c][:, None, None, :]


def _axis_weights(t, p, dmax):
    """[d][axis] -> (N, p) arrays of d-th derivative weights, d = 0..dmax."""
    return [[bspline(t[:, ax, :], p, d) for ax in range(3)] for d in range(dmax + 1)]


# ----------------------------------------------------------------------------
# 4. density (Eq. charge_dipole_assign)
# ----------------------------------------------------------------------------

def _spread_terms(pos, box, mesh, p, coeffs):
    """Assign sum_{abc} coeffs[(a,b,c)][i] * W_x^(a) W_y^(b) W_z^(c) of every atom.

    coeffs maps a derivative multi-index to a per-atom coefficient array.
    """
    M = int(np.prod(mesh))
    rho = np.zeros(M)
    dmax = max(sum(k) for k in coeffs)
    n = pos.shape[0]
    for s in range(0, n, _CHUNK):
        sl = slice(s, min(n, s + _CHUNK))
        idx, t = stencil(pos[sl], box, mesh, p)
        w = _axis_weights(t, p, dmax)
        wd = [[w[d][ax] for d in range(dmax + 1)] for ax in range(3)]
        val = np.zeros((idx.shape[0], p, p, p))
        for (a, b, c), coef in coeffs.items():
            val += coef[sl][:, None, None, None] * _w3(wd[0], wd[1], wd[2], a, b, c)
        rho += np.bincount(_flat(idx, mesh).ravel(), weights=val.ravel(), minlength=M)
    return rho.reshape(mesh)


def density(pos, q, mu, box, mesh, p):
    """rho(n) = sum_i sum_stencil [q W_xW_yW_z + sum_a N_a (mu . C^-1[:, a]) d_a W]."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    _, Cinv, _, _ = cell(box)
    N = np.asarray(mesh, dtype=np.float64)
    dip = N[None, :] * (mu @ Cinv)          # N_a (mu_i . C^-1[:, a])
    coeffs = {(0, 0, 0): q, (1, 0, 0): dip[:, 0], (0, 1, 0): dip[:, 1], (0, 0, 1): dip[:, 2]}
    return _spread_terms(pos, box, mesh, p, coeffs)


# ----------------------------------------------------------------------------
# 5-7. transform, influence function, potential (Eqs. fft, Bk, influence, green,
#      potential_k, ifft)
# ----------------------------------------------------------------------------

def dft_matrix(N: int, sign: int = -1) -> np.ndarray:
    k = np.arange(N)
    return np.exp(sign * 2j * math.pi * (np.outer(k, k) % N) / N)


def dft3(a, sign: int = -1):
    """Unnormalised 3D DFT sum_m a(m) exp(sign 2 pi i k.m/N) by DFT-matrix products."""
    a = np.asarray(a, dtype=np.complex128)
    Nx, Ny, Nz = a.shape
    a = a @ dft_matrix(Nz, sign).T                     # along z
    a = np.matmul(dft_matrix(Ny, sign), a)             # along y (batched over x)
    a = (dft_matrix(Nx, sign) @ a.reshape(Nx, -1)).reshape(Nx, Ny, Nz)
    return a


def signed_index(N: int) -> np.ndarray:
    """f = k - N [k >= ceil(N/2)], the fftfreq ordering (Nyquist at -N/2)."""
    k = np.arange(N)
    return k - N * (k >= (N + 1) // 2)


def influence_optimal(box, mesh, p, alpha, m_max=1):
    """The energy-optimal influence function of the assignment of order p, with
    aliasing sums (an alternative to the sinc^(-2 gamma p) deconvolution, Sec. 2.3.4
    mentions it only by name):
        g(f) = sum_m U^2(f + m N) G(k(f + m N)) / (sum_m U^2(f + m N))^2,
        U(f) = prod_a sinc(f_a / N_a)^p,  m in [-m_max, m_max]^3,  g(0) = 0.
    Restricted to m = 0 it is G / U^2, the gamma = 1 deconvolution."""
    _, _, _, recip = cell(box)
    N = [int(n) for n in mesh]
    f = [signed_index(n).astype(np.float64) for n in N]
    # separable denominator: sum_m U^2 = prod_a sum_{m_a} sinc^(2p)((f_a + m_a N_a)/N_a)
    S = [sum(np.sinc((f[a] + m * N[a]) / N[a]) ** (2 * p) for m in range(-m_max, m_max + 1))
         for a in range(3)]
    den = (S[0][:, None, None] * S[1][None, :, None] * S[2][None, None, :]) ** 2
    num = np.zeros(tuple(N))
    for mx in range(-m_max, m_max + 1):
        for my in range(-m_max, m_max + 1):
            for mz in range(-m_max, m_max + 1):
                fx, fy, fz = f[0] + mx * N[0], f[1] + my * N[1], f[2] + mz * N[2]
                u2 = (np.sinc(fx / N[0])[:, None, None] * np.sinc(fy / N[1])[None, :, None]
                      * np.sinc(fz / N[2])[None, None, :]) ** (2 * p)
                kvec = (fx[:, None, None, None] * recip[0] + fy[None, :, None, None] * recip[1]
                        + fz[None, None, :, None] * recip[2])
                k2 = np.einsum('xyzc,xyzc->xyz', kvec, kvec)
                with np.errstate(divide='ignore', invalid='ignore'):
                    G = 4.0 * math.pi / k2 * np.exp(-k2 / (4.0 * alpha * alpha))
                G[k2 == 0.0] = 0.0
                num += u2 * G
    g = num / den
    g[0, 0, 0] = 0.0
    return g


def influence(box, mesh, p, alpha, gamma=1.0):
    """g(n) = G(k) * C(n) on the full grid, with k = sum_a f_a b_a and g(0) = 0.
    gamma = "optimal" selects the energy-optimal influence function instead."""
    if isinstance(gamma, str):
        if gamma != "optimal":
            raise ValueError(gamma)
        return influence_optimal(box, mesh, p, alpha)
    _, _, _, recip = cell(box)
    fx, fy, fz = (signed_index(N).astype(np.float64) for N in mesh)
    kvec = (fx[:, None, None, None] * recip[0] + fy[None, :, None, None] * recip[1]
            + fz[None, None, :, None] * recip[2])
    k2 = np.einsum('xyzc,xyzc->xyz', kvec, kvec)
    with np.errstate(divide='ignore', invalid='ignore'):
        G = 4.0 * math.pi / k2 * np.exp(-k2 / (4.0 * alpha * alpha))
    G[0, 0, 0] = 0.0
    B = (np.sinc(fx / mesh[0])[:, None, None] ** p * np.sinc(fy / mesh[1])[None, :, None] ** p
         * np.sinc(fz / mesh[2])[None, None, :] ** p)
    return G / np.abs(B) ** (2.0 * gamma)


def potential(rho, g):
    """phi = Re IDFT[g * DFT[rho]] with an unnormalised inverse transform."""
    return dft3(g * dft3(rho, -1), +1).real


# ----------------------------------------------------------------------------
# 8-9. energy, gradients, Hessian-vector product
# ----------------------------------------------------------------------------

@dataclass
class PMEResult:
    e_recip: float
    e_self_q: float
    e_self_mu: float
    dE_dpos: np.ndarray
    dE_dq: np.ndarray
    dE_dmu: np.ndarray
    rho: np.ndarray
    phi: np.ndarray

    @property
    def energy(self) -> float:
        return self.e_recip + self.e_self_q + self.e_self_mu


def _stencil_sums(pos, box, mesh, p, field, orders):
    """S[(a,b,c)][i] = sum over atom i's stencil of field * W_x^(a) W_y^(b) W_z^(c)."""
    n = pos.shape[0]
    dmax = max(sum(k) for k in orders)
    out = {k: np.zeros(n) for k in orders}
    flatfield = np.asarray(field).ravel()
    for s in range(0, n, _CHUNK):
        sl = slice(s, min(n, s + _CHUNK))
        idx, t = stencil(pos[sl], box, mesh, p)
        w = _axis_weights(t, p, dmax)
        wd = [[w[d][ax] for d in range(dmax + 1)] for ax in range(3)]
        fv = flatfield[_flat(idx, mesh)]
        for key in orders:
            out[key][sl] = np.einsum('nijk,nijk->n', fv, _w3(wd[0], wd[1], wd[2], *key))
    return out


def _orders(deg):
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1) for c in range(deg + 1)
            if a + b + c == deg]


def _grad_vec(S):
    return np.stack([S[(1, 0, 0)], S[(0, 1, 0)], S[(0, 0, 1)]], axis=1)


def _hess_mat(S):
    H = np.empty((len(S[(2, 0, 0)]), 3, 3))
    for a in range(3):
        for b in range(3):
            key = [0, 0, 0]
            key[a] += 1
            key[b] += 1
            H[:, a, b] = S[tuple(key)]
    return H


def _third_contract(S, u, v):
    """out[i, c] = sum_{a,b} T[i,a,b,c] u[i,a] v[i,b] for the symmetric third-order sums."""
    out = np.zeros_like(u)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                key = [0, 0, 0]
                key[a] += 1
                key[b] += 1
                key[c] += 1
                out[:, c] += S[tuple(key)] * u[:, a] * v[:, b]
    return out


def _inputs(pos, q, mu):
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    q = np.zeros(n) if q is None else np.asarray(q, dtype=np.float64)
    mu = np.zeros((n, 3)) if mu is None else np.asarray(mu, dtype=np.float64)
    return pos, q, mu


def forward(pos, q, mu, box, mesh, p, alpha, gamma=1.0, prefactor=1.0) -> PMEResult:
    """E^lr and its gradients (Eqs. energy_recip, self_q, self_mu, E_lr_total, forces)."""
    pos, q, mu = _inputs(pos, q, mu)
    mesh = tuple(int(m) for m in mesh)
    _, _, V, _ = cell(box)
    J = jacobian(box, mesh)
    rho = density(pos, q, mu, box, mesh, p)
    phi = potential(rho, influence(box, mesh, p, alpha, gamma))
    e_recip = float(np.sum(rho * phi)) / (2.0 * V)
    e_self_q = -alpha / math.sqrt(math.pi) * float(np.sum(q * q))
    e_self_mu = -2.0 * alpha ** 3 / (3.0 * math.sqrt(math.pi)) * float(np.sum(mu * mu))
    S = _stencil_sums(pos, box, mesh, p, phi, _orders(0) + _orders(1) + _orders(2))
    g1 = _grad_vec(S)                    # sum phi grad_x W
    H = _hess_mat(S)                     # sum phi grad_x grad_x W
    d = mu @ J.T                         # J mu  (x-space dipole)
    dE_dq = S[(0, 0, 0)] / V - 2.0 * alpha / math.sqrt(math.pi) * q
    dE_dmu = (g1 @ J) / V - 4.0 * alpha ** 3 / (3.0 * math.sqrt(math.pi)) * mu
    dE_dpos = (q[:, None] * g1 + np.einsum('nab,nb->na', H, d)) @ J / V
    return PMEResult(prefactor * e_recip, prefactor * e_self_q, prefactor * e_self_mu,
                     prefactor * dE_dpos, prefactor * dE_dq, prefactor * dE_dmu, rho, phi)


def energy(pos, q, mu, box, mesh, p, alpha, gamma=1.0, prefactor=1.0) -> float:
    pos, q, mu = _inputs(pos, q, mu)
    _, _, V, _ = cell(box)
    rho = density(pos, q, mu, box, mesh, p)
    phi = potential(rho, influence(box, mesh, p, alpha, gamma))
    e = float(np.sum(rho * phi)) / (2.0 * V)
    e -= alpha / math.sqrt(math.pi) * float(np.sum(q * q))
    e -= 2.0 * alpha ** 3 / (3.0 * math.sqrt(math.pi)) * float(np.sum(mu * mu))
    return prefactor * e


def cell_gradient(pos, q, mu, box, mesh, p, alpha, gamma=1.0, prefactor=1.0) -> np.ndarray:
    """d E^lr / d C at fixed Cartesian positions, charges and dipoles (3x3, laid out
    like the box: G[a, b] = dE / dC[a, b]); what autograd of the pipeline gives for
    the cell (Sec. 2.4, the virial/stress loss).

    The self terms do not depend on C.  E_recip = (1/2V) sum_f g(f) |rho~(f)|^2
    depends on C through
      (i)   the volume:                     -E_recip C^-T
      (ii)  k = 2 pi C^-1 f in G(k) (the deconvolution depends on f alone), with
            dG/d(k^2) = -G (1/k^2 + 1/(4 alpha^2)) and d(k^2)/dC = -2 (C^-T k) k^T:
                                            (1/V) sum_f |rho~|^2 g (1/k^2 + 1/(4 alpha^2)) (C^-T k) k^T
      (iii) the density, whose mesh coordinates x_i = N (r_i C^-1) and x-space
            dipoles N (mu_i C^-1) move with C; with G_i = sum phi grad_x W and
            H_i = sum phi grad_x grad_x W over atom i's stencil and the unwrapped
            fractional coordinates s_i = r_i C^-1:
                                            -(1/V) [sum_i s_i (x) N (q_i G_i + H_i J mu_i)
                                                    + (mu_i C^-1) (x) N G_i] C^-T
    """
    if isinstance(gamma, str):
        raise NotImplementedError("the cell gradient is defined for the deconvolution influence")
    pos, q, mu = _inputs(pos, q, mu)
    mesh = tuple(int(m) for m in mesh)
    _, Cinv, V, recip = cell(box)
    J = jacobian(box, mesh)
    g = influence(box, mesh, p, alpha, gamma)
    rho = density(pos, q, mu, box, mesh, p)
    rk = dft3(rho, -1)
    phi = dft3(g * rk, +1).real
    e_recip = float(np.sum(rho * phi)) / (2.0 * V)
    # (ii)
    fx, fy, fz = (signed_index(N).astype(np.float64) for N in mesh)
    kvec = (fx[:, None, None, None] * recip[0] + fy[None, :, None, None] * recip[1]
            + fz[None, None, :, None] * recip[2])
    k2 = np.einsum('xyzc,xyzc->xyz', kvec, kvec)
    with np.errstate(divide='ignore', invalid='ignore'):
        fac = g * (1.0 / k2 + 1.0 / (4.0 * alpha * alpha))
    fac[0, 0, 0] = 0.0
    T = np.einsum('xyz,xyzc,xyzd->cd', np.abs(rk) ** 2 * fac, kvec, kvec)
    term2 = Cinv.T @ T / V
    # (iii)
    S = _stencil_sums(pos, box, mesh, p, phi, _orders(1) + _orders(2))
    G, H = _grad_vec(S), _hess_mat(S)
    gx = q[:, None] * G + np.einsum('nab,nb->na', H, mu @ J.T)
    Nv = np.asarray(mesh, dtype=np.float64)
    s = pos @ Cinv
    term3 = -((s.T @ (gx * Nv)) + ((mu @ Cinv).T @ (G * Nv))) @ Cinv.T / V
    term1 = -e_recip * Cinv.T
    return prefactor * (term1 + term2 + term3)


def hvp(pos, q, mu, box, mesh, p, alpha, v_pos=None, v_q=None, v_mu=None, gamma=1.0,
        prefactor=1.0):
    """Hessian of E^lr in (r, q, mu) applied to (v_pos, v_q, v_mu).

    With rho_i = q_i W_i + mu_i . D_i (D_i = grad_r W_i, H_i = grad_r grad_r W_i):
      tangent density  rho_dot = sum_i [v_q W + (v_mu + q v_r) . D + mu^T H v_r]
      psi = K rho_dot  (same mesh operator as the potential)
      q_bar  = (1/V) sum [W psi + (D . v_r) phi]                - 2a/sqrt(pi) v_q
      mu_bar = (1/V) sum [D psi + H v_r phi]                    - 4a^3/(3 sqrt(pi)) v_mu
      r_bar  = (1/V) sum [(q D + H mu) psi
                          + (v_q D + H (v_mu + q v_r) + grad_r(mu^T H v_r)) phi]
    """
    pos, q, mu = _inputs(pos, q, mu)
    n = pos.shape[0]
    v_pos = np.zeros((n, 3)) if v_pos is None else np.asarray(v_pos, dtype=np.float64)
    v_q = np.zeros(n) if v_q is None else np.asarray(v_q, dtype=np.float64)
    v_mu = np.zeros((n, 3)) if v_mu is None else np.asarray(v_mu, dtype=np.float64)
    mesh = tuple(int(m) for m in mesh)
    _, _, V, _ = cell(box)
    J = jacobian(box, mesh)
    g = influence(box, mesh, p, alpha, gamma)
    phi = potential(density(pos, q, mu, box, mesh, p), g)

    d = mu @ J.T                                  # J mu
    vh = v_pos @ J.T                              # J v_r
    wh = (v_mu + q[:, None] * v_pos) @ J.T        # J (v_mu + q v_r)
    coeffs = {(0, 0, 0): v_q}
    for a, key in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        coeffs[key] = wh[:, a]
    for a in range(3):
        for b in range(3):
            key = [0, 0, 0]
            key[a] += 1
            key[b] += 1
            key = tuple(key)
            coeffs[key] = coeffs.get(key, 0.0) + d[:, a] * vh[:, b]
    rho_dot = _spread_terms(pos, box, mesh, p, coeffs)
    psi = potential(rho_dot, g)

    P = _stencil_sums(pos, box, mesh, p, psi, _orders(0) + _orders(1) + _orders(2))
    S = _stencil_sums(pos, box, mesh, p, phi, _orders(1) + _orders(2) + _orders(3))
    P1, P2 = _grad_vec(P), _hess_mat(P)
    S1, S2 = _grad_vec(S), _hess_mat(S)
    c_q = 2.0 * alpha / math.sqrt(math.pi)
    c_mu = 4.0 * alpha ** 3 / (3.0 * math.sqrt(math.pi))
    g_q = (P[(0, 0, 0)] + np.sum(S1 * vh, axis=1)) / V - c_q * v_q
    g_mu = (P1 + np.einsum('nab,nb->na', S2, vh)) @ J / V - c_mu * v_mu
    rx = (q[:, None] * P1 + np.einsum('nab,nb->na', P2, d) + v_q[:, None] * S1
          + np.einsum('nab,nb->na', S2, wh) + _third_contract(S, d, vh))
    g_pos = rx @ J / V
    return prefactor * g_pos, prefactor * g_q, prefactor * g_mu
