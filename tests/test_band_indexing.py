"""Host check of the band spread's integer logic (k_spread_band): for every x-plane and
band of small meshes, every order 1-7 and every bin size that divides the mesh, the
scanned bin runs hold every anchor whose stencil reaches the plane and the band, the
hit test on an anchor's first stencil row equals "some stencil row lies in the band",
and the rows an atom adds are exactly its stencil rows inside the band.  The index
expressions are restated here from the kernel; brute force over the stencil is the
reference."""
import itertools

import pytest


def bin_run(first, length, n, b, nb):
    # bins along one axis whose anchors lie in the cyclic range [first, first + length)
    if length >= n:
        return 0, nb
    lo, hi = first % n, (first + length - 1) % n
    k0, k1 = lo // b, hi // b
    if lo + length - 1 < n:
        cnt = k1 - k0 + 1
    else:
        cnt = nb - k0 + k1 + 1 if k1 < k0 else nb
    return k0, min(cnt, nb)


def band_rows(ny, rows_max):
    nband = -(-ny // rows_max)
    return -(-ny // nband), nband


@pytest.mark.parametrize("p", range(1, 8))
def test_band_indexing_matches_brute_force(p):
    lo = (p - 1) // 2
    checked = 0
    for nx, ny, bsz, rows_max in itertools.product((8, 12, 15), (9, 16, 21), (2, 3, 4, 5),
                                                   (4, 7, 64)):
        if nx % bsz or ny % bsz or nx < p + bsz or ny < p + bsz:
            continue
        nbx, nby = nx // bsz, ny // bsz
        rows, nband = band_rows(ny, rows_max)
        assert (nband - 1) * rows < ny <= nband * rows
        for x in range(nx):
            k0, nl = bin_run(x + lo - p + 1, p, nx, bsz, nbx)
            layers = {(k0 + i) % nbx for i in range(nl)}
            for bx in range(nx):
                if (x - bx + lo) % nx < p:           # the x stencil reaches plane x
                    assert bx // bsz in layers
        for band in range(nband):
            y0 = band * rows
            nrows = min(rows, ny - y0)
            ky0, nly = bin_run(y0 + lo - p + 1, nrows + p - 1, ny, bsz, nby)
            ybins = {(ky0 + i) % nby for i in range(nly)}
            for by in range(ny):
                stencil = {(by - lo + j) % ny for j in range(p)}
                inside = {r - y0 for r in stencil if y0 <= r < y0 + nrows}
                t = (by - lo - y0) % ny                  # first stencil row, band-relative
                hit = t < nrows or t + p - 1 >= ny
                assert hit == bool(inside), (p, ny, rows, band, by)
                if inside:
                    assert by // bsz in ybins
                added = set()
                for iy in range(p):
                    rr = t + iy
                    rr -= ny if rr >= ny else 0
                    if rr < nrows:
                        added.add(rr)
                assert added == inside
                checked += 1
    assert checked > 0
