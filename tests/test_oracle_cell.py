"""Pins of the oracle's cell gradient dE^lr/dC at fixed Cartesian inputs (the
stress/virial loss of Sec. 2.4; CPU only), each against something other than
the formula it implements:

* central finite differences of the oracle's own energy along every entry of a
  triclinic cell, with atoms outside the cell (unwrapped positions);
* the exact rotation identity: E^lr is unchanged when the cell, positions and
  dipoles are rotated together, so C^T dE/dC + sum_i r_i (x) dE/dr_i +
  sum_i mu_i (x) dE/dmu_i is a symmetric matrix;
* the exact lattice-image identity: moving atom i by the lattice vector n C
  leaves E^lr unchanged for every C, so dE/dC changes by -n (x) dE/dr_i;
* convergence, as the mesh and order are raised, to central differences of the
  explicit Ewald reciprocal + self energy (a different method).
"""
import numpy as np
import pytest

import synth
from oracle import ewald, pme


def _fd_cell(energy, box, h=1e-5):
    out = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            bp = box.copy()
            bm = box.copy()
            bp[i, j] += h
            bm[i, j] -= h
            out[i, j] = (energy(bp) - energy(bm)) / (2.0 * h)
    return out


def _frame(n, seed, charges=True, dipoles=True):
    rng = np.random.default_rng(seed)
    box = np.array([[10.0, 0.3, -0.2], [0.5, 11.0, 0.4], [-0.3, 0.6, 9.5]])
    pos = rng.uniform(-2.0, 12.0, (n, 3))          # some atoms outside the cell
    q = rng.normal(0.0, 1.0, n) if charges else np.zeros(n)
    q -= q.mean()
    mu = rng.normal(0.0, 0.3, (n, 3)) if dipoles else np.zeros((n, 3))
    return pos, q, mu, box


@pytest.mark.parametrize("p,mesh", [(5, (12, 14, 13)), (6, (16, 15, 12)), (4, (10, 12, 11))])
def test_cell_gradient_finite_difference(p, mesh):
    pos, q, mu, box = _frame(30, 3 + p)
    a = 0.35
    g = pme.cell_gradient(pos, q, mu, box, mesh, p, a, prefactor=1.7)
    fd = _fd_cell(lambda b: pme.energy(pos, q, mu, b, mesh, p, a, prefactor=1.7), box)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max()


@pytest.mark.parametrize("charges,dipoles", [(True, True), (True, False), (False, True)])
def test_cell_gradient_rotation_identity(charges, dipoles):
    pos, q, mu, box = _frame(40, 11, charges, dipoles)
    mesh, p, a = (14, 15, 13), 6, 0.3
    g = pme.cell_gradient(pos, q, mu, box, mesh, p, a)
    r = pme.forward(pos, q, mu, box, mesh, p, a)
    W = box.T @ g + pos.T @ r.dE_dpos + mu.T @ r.dE_dmu
    assert np.abs(W - W.T).max() <= 1e-12 * np.abs(W).max()
    # and a dropped term or a transposed factor breaks it
    assert np.abs(g - g.T).max() > 1e-6 * np.abs(g).max()


def test_cell_gradient_lattice_image_shift():
    pos, q, mu, box = _frame(20, 5)
    mesh, p, a = (12, 12, 12), 5, 0.4
    g0 = pme.cell_gradient(pos, q, mu, box, mesh, p, a)
    f0 = pme.forward(pos, q, mu, box, mesh, p, a).dE_dpos
    n = np.array([1.0, -2.0, 1.0])
    moved = pos.copy()
    moved[7] += n @ box
    g1 = pme.cell_gradient(moved, q, mu, box, mesh, p, a)
    want = g0 - np.outer(n, f0[7])
    assert np.abs(g1 - want).max() <= 1e-10 * np.abs(g0).max()


def test_cell_gradient_converges_to_ewald():
    f = synth.triclinic_cell()
    a = 0.45
    ref = _fd_cell(lambda b: ewald.ewald_long_range(f.pos, f.q, f.mu, b, a)[0], f.box)
    errs = []
    for p, spacing in [(5, 1.0), (6, 0.7), (7, 0.5)]:
        mesh = pme.mesh_dims(f.box, spacing, "smooth")
        g = pme.cell_gradient(f.pos, f.q, f.mu, f.box, mesh, p, a)
        errs.append(np.abs(g - ref).max() / np.abs(ref).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[-1] < 1e-7
