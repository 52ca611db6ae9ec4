"""Pins of the oracle's assignment weights and discrete transform (CPU only).

The weights follow Sec. 2.3.2 (W^(p) read as the centered cardinal B-spline,
whose transform is the sinc^p response of Eq. Bk).  They are pinned by exact
rationals, by an independent library evaluation (scipy's B-spline basis
element built by de Boor's recursion), by the partition of unity and moment
identities, and by the Fourier response.  The DFT-matrix transform used for
Eq. fft is pinned by the literal triple sum and by numpy's FFT.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import pme
from oracle.bspline import bspline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "bspline_values.txt")):
        if line.startswith("#") or not line.strip():
            continue
        p, t, a, b = line.split()
        rows.append((int(p), float(t), int(a) / int(b)))
    return rows


@pytest.mark.parametrize("p,t,val", _golden_rows())
def test_bspline_exact_rationals(p, t, val):
    assert bspline(np.array([t]), p)[0] == pytest.approx(val, rel=1e-14, abs=1e-16)


@pytest.mark.parametrize("p", range(1, 8))
def test_bspline_matches_de_boor(p):
    # avoid the knots, where the highest derivative is only defined one-sidedly
    t = np.linspace(-p / 2 - 0.5, p / 2 + 0.5, 997) + 1e-3
    ref = BSpline.basis_element(np.arange(p + 1) - p / 2, extrapolate=False)
    for d in range(0, min(p, 4)):
        r = np.nan_to_num((ref.derivative(d) if d else ref)(t))
        assert np.max(np.abs(r - bspline(t, p, d))) < 1e-11


@pytest.mark.parametrize("p", range(1, 8))
def test_partition_of_unity_and_moments(p):
    rng = np.random.default_rng(p)
    for x in rng.uniform(-5, 5, 25):
        m = np.arange(math.floor(x) - 5, math.floor(x) + 6)
        w = bspline(x - m, p)
        assert np.sum(w) == pytest.approx(1.0, abs=1e-11)
        if p >= 2:
            assert np.sum(m * w) == pytest.approx(x, abs=1e-10)
            assert np.sum(bspline(x - m, p, 1)) == pytest.approx(0.0, abs=1e-10)
        if p >= 3:
            # second moment of M_p about x is p/12 (variance of p uniform variables)
            assert np.sum((m - x) ** 2 * w) == pytest.approx(p / 12.0, abs=1e-10)


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7])
def test_derivatives_are_finite_differences(p):
    t = np.linspace(-p / 2 + 0.013, p / 2 - 0.011, 301)
    h = 1e-5
    for d in range(1, p - 1):
        fd = (bspline(t + h, p, d - 1) - bspline(t - h, p, d - 1)) / (2 * h)
        assert np.max(np.abs(fd - bspline(t, p, d))) < 1e-7 * max(1.0, np.max(np.abs(fd)))


@pytest.mark.parametrize("p", [2, 4, 6, 7])
def test_fourier_response_is_sinc_power(p):
    # the continuous transform of M_p is sinc^p (the response of Eq. Bk)
    t = np.linspace(-p / 2, p / 2, 20001)
    w = bspline(t, p)
    for f in (0.1, 0.25, 0.4):
        ft = np.trapezoid(w * np.cos(2 * math.pi * f * t), t)
        assert ft == pytest.approx(np.sinc(f) ** p, abs=1e-7)


def test_stencil_weight_sums():
    """Each atom's stencil weights sum to 1 and its dipole weights to 0 (any p)."""
    rng = np.random.default_rng(3)
    pos = rng.uniform(-3, 20, (50, 3))
    box = np.diag([9.0, 10.0, 11.0])
    for p in range(1, 8):
        idx, t = pme.stencil(pos, box, (9, 10, 11), p)
        w = bspline(t, p)
        assert np.allclose(w.sum(axis=2), 1.0, atol=1e-13)
        assert np.all(np.abs(t) <= p / 2 + 1e-12)
        if p >= 2:
            assert np.allclose(bspline(t, p, 1).sum(axis=2), 0.0, atol=1e-12)


def _literal_dft(a, sign):
    Nx, Ny, Nz = a.shape
    out = np.zeros(a.shape, dtype=complex)
    for k in itertools.product(range(Nx), range(Ny), range(Nz)):
        s = 0j
        for m in itertools.product(range(Nx), range(Ny), range(Nz)):
            ph = k[0] * m[0] / Nx + k[1] * m[1] / Ny + k[2] * m[2] / Nz
            s += a[m] * complex(math.cos(2 * math.pi * ph), sign * math.sin(2 * math.pi * ph))
        out[k] = s
    return out


@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 4, 3), (6, 5, 6)])
def test_dft_matches_literal_triple_sum(shape):
    rng = np.random.default_rng(sum(shape))
    a = rng.normal(size=shape)
    for sign in (-1, +1):
        assert np.allclose(pme.dft3(a, sign), _literal_dft(a, sign), atol=1e-11)


def test_dft_library_crosscheck_and_special_cases():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(8, 10, 12))
    assert np.allclose(pme.dft3(a, -1), np.fft.fftn(a), atol=1e-10)
    assert np.allclose(pme.dft3(a, +1), np.fft.ifftn(a) * a.size, atol=1e-10)
    delta = np.zeros((6, 5, 4))
    delta[0, 0, 0] = 1.0
    assert np.allclose(pme.dft3(delta), 1.0)
    m = np.indices((6, 5, 4))
    wave = np.exp(2j * math.pi * (2 * m[0] / 6 + 1 * m[1] / 5 + 3 * m[2] / 4))
    spec = pme.dft3(wave)
    expect = np.zeros((6, 5, 4), dtype=complex)
    expect[2, 1, 3] = 120.0
    assert np.allclose(spec, expect, atol=1e-10)


def test_signed_index_is_fftfreq_order():
    for N in (1, 2, 5, 6, 16, 25, 100):
        assert np.array_equal(pme.signed_index(N), np.round(np.fft.fftfreq(N) * N).astype(int))


def test_mesh_dims_strategies():
    box = np.diag([10.0, 11.3, 7.9])
    # targets ceil(2|a|/Delta + 1) with Delta = 1: 21, 24 (23.6), 17 (16.8)
    assert pme.mesh_dims(box, 1.0, "ceil") == (21, 24, 17)
    assert pme.mesh_dims(box, 1.0, "smooth") == (24, 24, 18)
    assert pme.mesh_dims(box, 1.0, "pow2") == (32, 32, 32)
