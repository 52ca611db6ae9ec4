"""pme_forward_noalloc (no plan, fixed scratch array per GPU) against pme_forward
on a plan, through the C ABI: two calls in a row, the second with a smaller input
(fewer atoms, smaller mesh, other order), each to the parity bar (1e-5 relative
energy, 1e-4 relative RMS per-atom gradients); the first also against the oracle.
Host-side rejections (workspace above the scratch array, optimal influence) are
checked too."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_util import E_REL_TOL, RMS_REL_TOL, dev, host, oracle_forward, rel, rms_rel, to_dev

pytestmark = pytest.mark.gpu


def _desc(mesh, p, alpha, max_atoms=1, flags=0):
    from paper_2606_01598_amd import _lib
    d = _lib.PMEDesc()
    for k in range(3):
        d.mesh[k] = int(mesh[k])
        d.tile[k] = 0
    d.order = int(p)
    d.max_atoms = int(max_atoms)
    d.flags = int(flags)
    d.alpha = float(alpha)
    d.influence_power = 1.0
    d.prefactor = 1.0
    return d


def _noalloc(frame, mesh, p, alpha):
    from paper_2606_01598_amd import _lib
    lib = _lib.load()
    pos, q, mu, box = to_dev(frame)
    n = frame.n
    out = {"energy": torch.full((3,), float("nan"), dtype=torch.float64, device=dev()),
           "dE_dpos": torch.full((n, 3), float("nan"), device=dev()),
           "dE_dq": torch.full((n,), float("nan"), device=dev()),
           "dE_dmu": torch.full((n, 3), float("nan"), device=dev())}
    d = _desc(mesh, p, alpha)
    s = torch.cuda.current_stream().cuda_stream
    rc = lib.pme_forward_noalloc(ctypes.byref(d), s, n, pos.data_ptr(), q.data_ptr(),
                                 mu.data_ptr(), box.data_ptr(), out["energy"].data_ptr(),
                                 out["dE_dpos"].data_ptr(), out["dE_dq"].data_ptr(),
                                 out["dE_dmu"].data_ptr())
    _lib.check(rc)
    torch.cuda.synchronize()
    return out


def _plan_forward(frame, mesh, p, alpha):
    from paper_2606_01598_amd.pme import Plan
    plan = Plan(mesh, p, alpha, max_atoms=frame.n)
    out = plan.forward(*to_dev(frame))
    plan.status()
    return out


def _compare(label, got, ref):
    errs = {"energy": rel(host(got["energy"]).sum(), host(ref["energy"]).sum())}
    for k in ("dE_dpos", "dE_dq", "dE_dmu"):
        errs[k] = rms_rel(host(got[k]), host(ref[k]))
    bitwise = all(torch.equal(got[k], ref[k]) for k in ref)
    print(label, "bitwise", bitwise, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["energy"] <= E_REL_TOL
    assert max(v for k, v in errs.items() if k != "energy") <= RMS_REL_TOL
    return bitwise


def test_noalloc_forward_two_calls_second_smaller():
    print("case: pme_forward_noalloc 1000 ions 32^3 p=6, then 300 ions 24^3 p=5", flush=True)
    f1 = synth.molten_box(1000, 1, L=31.5)
    got1 = _noalloc(f1, (32, 32, 32), 6, 0.3)
    ref1 = _plan_forward(f1, (32, 32, 32), 6, 0.3)
    _compare("call 1", got1, ref1)
    o = oracle_forward(f1, (32, 32, 32), 6, 0.3)
    assert rel(host(got1["energy"]).sum(), o.energy) <= E_REL_TOL
    assert rms_rel(host(got1["dE_dpos"]), o.dE_dpos) <= RMS_REL_TOL
    f2 = synth.molten_box(300, 2, L=21.0)
    got2 = _noalloc(f2, (24, 24, 24), 5, 0.35)
    ref2 = _plan_forward(f2, (24, 24, 24), 5, 0.35)
    _compare("call 2 (smaller)", got2, ref2)


def test_noalloc_host_rejections():
    from paper_2606_01598_amd import _lib
    lib = _lib.load()
    f = synth.molten_box(100, 3, L=15.0)
    pos, q, mu, box = to_dev(f)
    e = torch.empty(3, dtype=torch.float64, device=dev())
    s = torch.cuda.current_stream().cuda_stream
    args = (s, f.n, pos.data_ptr(), q.data_ptr(), mu.data_ptr(), box.data_ptr(), e.data_ptr(),
            None, None, None)
    big = _desc((512, 512, 512), 6, 0.3)
    assert lib.pme_forward_noalloc(ctypes.byref(big), *args) == _lib.PME_ESCRATCH
    opt = _desc((16, 16, 16), 6, 0.3, flags=_lib.PME_F_OPT_INFLUENCE)
    assert lib.pme_forward_noalloc(ctypes.byref(opt), *args) == _lib.PME_EINVAL
    assert lib.pme_forward_noalloc(None, *args) == _lib.PME_EINVAL


def test_noalloc_forward_band_mesh():
    # a mesh whose padded y-z plane does not fit beside the slab transform: the
    # band spread, in the fixed scratch array as in a plan
    from paper_2606_01598_amd.pme import Plan
    mesh, p, alpha = (24, 128, 120), 6, 0.3
    print(f"case: pme_forward_noalloc band mesh {mesh} p={p}", flush=True)
    rng = np.random.default_rng(31)
    n = 2000
    diag = np.array([24.0, 128.0, 120.0])
    f = synth.Frame(pos=rng.uniform(0.0, 1.0, (n, 3)) * diag,
                    q=np.where(np.arange(n) % 2 == 0, 1.0, -1.0),
                    mu=rng.normal(0.0, 0.1, (n, 3)), box=np.diag(diag))
    got = _noalloc(f, mesh, p, alpha)   # before any plan: the entry point's own set-up
    assert Plan(mesh, p, alpha, max_atoms=n).spread_kind == "band"
    ref = _plan_forward(f, mesh, p, alpha)
    assert _compare("band mesh", got, ref)
    o = oracle_forward(f, mesh, p, alpha)
    assert rel(host(got["energy"]).sum(), o.energy) <= E_REL_TOL
    assert rms_rel(host(got["dE_dpos"]), o.dE_dpos) <= RMS_REL_TOL
