"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, maps return codes to text, computes mesh dimensions (Eq.
mesh_target and the three strategies of Sec. 2.3.1) like the oracle, and
rejects invalid plan descriptors before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import pme as opme
from paper_2606_01598_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpme.so is not built: run `python -m paper_2606_01598_amd.build`")
    return _lib.load()


def test_header_declarations_are_exported():
    lib = _lib_or_skip()
    declared = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            declared |= set(re.findall(r"\b((?:pme|pol|dip)_[a-z_0-9]+)\s*\(", text))
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_strerror_codes():
    lib = _lib_or_skip()
    for code in range(-9, 1):
        assert lib.pme_strerror(code).decode() != "unknown error"
    assert lib.pme_strerror(-99).decode() == "unknown error"


@pytest.mark.parametrize("strategy,code", [("pow2", 0), ("smooth", 1), ("ceil", 2)])
def test_mesh_dims_matches_oracle(strategy, code):
    lib = _lib_or_skip()
    rng = np.random.default_rng(4)
    for _ in range(20):
        box = np.diag(rng.uniform(5, 80, 3))
        box[1, 0] = rng.uniform(-2, 2)
        box[2, :2] = rng.uniform(-2, 2, 2)
        spacing = float(rng.uniform(0.3, 2.0))
        out = (ctypes.c_int32 * 3)()
        b = (ctypes.c_double * 9)(*box.ravel())
        assert lib.pme_mesh_dims(b, spacing, code, out) == 0
        assert tuple(out) == opme.mesh_dims(box, spacing, strategy)


def test_mesh_dims_rejects_bad_input():
    lib = _lib_or_skip()
    out = (ctypes.c_int32 * 3)()
    good = (ctypes.c_double * 9)(*np.eye(3).ravel() * 10)
    sing = (ctypes.c_double * 9)(*np.zeros(9))
    assert lib.pme_mesh_dims(good, 0.0, 1, out) == _lib.PME_EINVAL
    assert lib.pme_mesh_dims(good, 1.0, 7, out) == _lib.PME_EINVAL
    assert lib.pme_mesh_dims(sing, 1.0, 1, out) == _lib.PME_EINVAL


def _desc(**kw):
    d = _lib.PMEDesc()
    mesh = kw.get("mesh", (16, 16, 16))
    for k in range(3):
        d.mesh[k] = mesh[k]
    d.order = kw.get("order", 4)
    d.max_atoms = kw.get("max_atoms", 64)
    d.flags = kw.get("flags", 0)
    d.alpha = kw.get("alpha", 0.3)
    d.influence_power = kw.get("gamma", 1.0)
    d.prefactor = kw.get("prefactor", 1.0)
    d.fft_lines = kw.get("fft_lines", 0)
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(order=0), _lib.PME_EORDER),
    (dict(order=8), _lib.PME_EORDER),
    (dict(mesh=(16, 16, 7)), _lib.PME_EMESH),
    (dict(mesh=(1, 16, 16)), _lib.PME_EMESH),
    (dict(mesh=(16, 2048, 16)), _lib.PME_EMESH),
    (dict(alpha=0.0), _lib.PME_EALPHA),
    (dict(alpha=float("nan")), _lib.PME_EALPHA),
    (dict(gamma=-1.0), _lib.PME_EALPHA),
    (dict(prefactor=float("inf")), _lib.PME_EALPHA),
    (dict(max_atoms=0), _lib.PME_EINVAL),
    (dict(flags=16), _lib.PME_EINVAL),
    (dict(fft_lines=-1), _lib.PME_EINVAL),
    (dict(fft_lines=1025), _lib.PME_EINVAL),
])
def test_plan_create_validation(kw, code):
    lib = _lib_or_skip()
    h = ctypes.c_void_p()
    d = _desc(**kw)
    assert lib.pme_plan(ctypes.byref(d), ctypes.byref(h)) == code
    assert not h.value


def test_null_arguments():
    lib = _lib_or_skip()
    h = ctypes.c_void_p()
    assert lib.pme_plan(None, ctypes.byref(h)) == _lib.PME_EINVAL
    assert lib.pme_forward(None, None, 0, None, None, None, None, None, None, None, None) == _lib.PME_EINVAL
    assert lib.pme_backward(None, None, 0, None, None, None, None, None, None, None, None, None,
                            None) == _lib.PME_EINVAL
    assert lib.pme_status(None, None) == _lib.PME_EINVAL
    lib.pme_plan_destroy(None)
    assert lib.pme_plan_workspace_bytes(None) == 0
    assert lib.pme_plan_spread_kind(None) == _lib.PME_EINVAL


def test_teacher_and_head_calls_reject_a_missing_plan():
    """The polarizable-model and learned-head calls check their arguments before
    touching the device: a NULL plan is PME_EINVAL."""
    lib = _lib_or_skip()
    E = _lib.PME_EINVAL
    n = 4
    assert lib.pol_real(None, None, n, *([None] * 8)) == E
    assert lib.pol_model(None, None, None, n, *([None] * 9)) == E
    assert lib.pol_model_hvp(None, None, None, n, *([None] * 10)) == E
    assert lib.dip_features(None, None, n, *([None] * 4)) == E
    assert lib.dip_features_jvp(None, None, n, *([None] * 6)) == E
    assert lib.dip_charges(None, None, n, *([None] * 6)) == E
    assert lib.dip_forward_jvp(None, None, n, *([None] * 7)) == E
    assert lib.dip_position_vjp(None, None, n, *([None] * 10)) == E
    assert lib.dip_backward_jvp(None, None, n, *([None] * 14)) == E
    assert lib.dip_loss(None, None, n, *([None] * 8), 1.0, 1.0, 0.0, *([None] * 4)) == E
    assert lib.dip_adam(None, 4, 0, 1e-3, 0.9, 0.999, 1e-8, None, None, None, None) == E


def test_learning_rate_schedule():
    """Adam's learning rate in the dipole-head trainer: a linear warmup over the
    first steps, then exponential decay (the optimizer setting of Sec. 2.4)."""
    from types import SimpleNamespace

    from paper_2606_01598_amd.dip import Trainer
    tr = SimpleNamespace(lr=1e-3, warmup=10, decay=0.5, decay_steps=100)
    rate = lambda t: Trainer.rate(tr, t)
    assert abs(rate(1) - 1e-4) < 1e-15 and abs(rate(5) - 5e-4) < 1e-15
    assert abs(rate(10) - 1e-3) < 1e-15
    assert abs(rate(110) - 5e-4) < 1e-15 and abs(rate(210) - 2.5e-4) < 1e-15
    tr0 = SimpleNamespace(lr=2e-3, warmup=0, decay=1.0, decay_steps=1)
    assert Trainer.rate(tr0, 1) == 2e-3 and Trainer.rate(tr0, 1000) == 2e-3


def test_halo_probe_rejects_bad_arguments():
    """pme_halo_probe validates on the host before any launch (no GPU needed)."""
    import ctypes
    lib = _lib_or_skip()
    N = (ctypes.c_int32 * 3)(100, 100, 100)
    T = (ctypes.c_int32 * 3)(10, 10, 20)
    buf = ctypes.c_void_p(16)   # never dereferenced on these paths
    cases = [
        (9, N, T, 6, buf, buf),                                   # unknown kind
        (_lib.PME_PROBE_HALO_WRITE, N, T, 6, None, buf),          # no region buffer
        (_lib.PME_PROBE_HALO_ATOMIC, N, T, 6, buf, None),         # no mesh
        (_lib.PME_PROBE_HALO_ATOMIC, N, (ctypes.c_int32 * 3)(10, 10, 30), 6, buf, buf),  # T does not divide N
        (_lib.PME_PROBE_HALO_ATOMIC, (ctypes.c_int32 * 3)(12, 12, 12), (ctypes.c_int32 * 3)(12, 12, 12),
         6, buf, buf),                                            # N < T + p - 1
        (_lib.PME_PROBE_HALO_FOLD, N, T, 0, buf, buf),            # order
    ]
    for kind, n, t, p, reg, mesh in cases:
        assert lib.pme_halo_probe(None, kind, n, t, p, reg, mesh) == _lib.PME_EINVAL


def test_batch_plan_rejects_mixed_influence_functions():
    # every box uses the optimal influence function or none; the check comes before
    # any device work
    lib = _lib_or_skip()
    descs = (_lib.PMEDesc * 2)(_desc(), _desc(flags=_lib.PME_F_OPT_INFLUENCE))
    n = (ctypes.c_int32 * 2)(10, 10)
    h = ctypes.c_void_p()
    assert lib.pme_batch_plan(descs, 2, n, ctypes.byref(h)) == _lib.PME_EINVAL
    assert not h.value
