"""The halo-combination probe (include/probe.h, pme_halo_probe) on small meshes:
the atomic combination and the region blocks folded per point give the same exact
counts, equal to the number of (T + p - 1)^3 regions that cover each mesh point,
computed here on the host from the region geometry."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _coverage(N, T, p):
    lo = (p - 1) // 2
    cov = []
    for a in range(3):
        c = np.zeros(N[a], dtype=np.int64)
        for k in range(N[a] // T[a]):
            for r in range(T[a] + p - 1):
                c[(k * T[a] - lo + r) % N[a]] += 1
        cov.append(c)
    return cov[0][:, None, None] * cov[1][None, :, None] * cov[2][None, None, :]


@pytest.mark.parametrize("N,T,p", [((24, 24, 24), (8, 8, 8), 6), ((30, 36, 40), (10, 12, 8), 4),
                                   ((20, 16, 18), (5, 8, 6), 2)])
def test_halo_probe_combinations_are_exact(N, T, p):
    from paper_2606_01598_amd import _lib
    lib = _lib.load()
    print(f"case: halo probe N={N} T={T} p={p}", flush=True)
    d = dev()
    tiles = np.prod([n // t for n, t in zip(N, T)])
    vol = np.prod([t + p - 1 for t in T])
    regions = torch.empty(int(tiles * vol), dtype=torch.int64, device=d)
    m64 = torch.zeros(int(np.prod(N)), dtype=torch.int64, device=d)
    m32 = torch.empty(int(np.prod(N)), dtype=torch.float32, device=d)
    cN = (ctypes.c_int32 * 3)(*N)
    cT = (ctypes.c_int32 * 3)(*T)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for kind, mesh in ((_lib.PME_PROBE_HALO_ATOMIC, m64), (_lib.PME_PROBE_HALO_WRITE, m64),
                       (_lib.PME_PROBE_HALO_FOLD, m32)):
        _lib.check(lib.pme_halo_probe(s, kind, cN, cT, p, ctypes.c_void_p(regions.data_ptr()),
                                      ctypes.c_void_p(mesh.data_ptr())))
    torch.cuda.synchronize()
    ref = _coverage(N, T, p).reshape(-1)
    assert np.array_equal(m64.cpu().numpy(), ref)
    assert np.array_equal(m32.cpu().numpy(), ref.astype(np.float32))
    assert int(ref.sum()) == tiles * vol
