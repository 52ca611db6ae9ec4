"""Oracle parity at the sizes the benchmark times, in the launch configuration it
times: pme_step with the cotangent chain on a second stream (PME_F_CONCURRENT),
eager and replayed from a captured HIP graph, on the molten-salt workloads of the
size sweep (Sec. 3.2 supercell scaling; synthetic stand-ins for its data):

* 32,000 ions on 100^3: every output of every atom against the oracle run here;
* 128,000 ions on 160^3 and 1,000,000 ions on 320^3 (the pencil FFT layout, with
  the x pass in column chunks of 4): the three energy terms and a seeded sample
  of 256 atoms against the values tests/golden/make_fullsize.py wrote with the
  oracle on every atom of the same seeded inputs.

Bar: 1e-5 relative energy (E_recip and E^lr), 1e-4 relative RMS for each
per-atom output (forces, dE/dq, dE/dmu and the three H v outputs).
"""
import os
import sys

import numpy as np
import pytest
import torch

import synth
from gpu_util import E_REL_TOL, RMS_REL_TOL, dev, f32, host, oracle_forward, oracle_hvp, rel, rms_rel

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize  # noqa: E402

KEYS = ("dE_dpos", "dE_dq", "dE_dmu", "g_pos", "g_q", "g_mu")
COLS = {"dE_dpos": slice(0, 3), "dE_dq": slice(3, 4), "dE_dmu": slice(4, 7),
        "g_pos": slice(7, 10), "g_q": slice(10, 11), "g_mu": slice(11, 14)}


def _inputs(n, seed):
    from paper_2606_01598_amd.pme import Plan  # noqa: F401  (fails loudly without the library)
    f = synth.molten_box(n, seed)
    v = synth.random_cotangents(n, make_fullsize.COT_SEED, scale_r=0.1)
    d = dev()
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=d)
    args = (t(f.pos), t(f.q), t(f.mu), torch.tensor(f.box, dtype=torch.float64, device=d))
    return f, v, args, [t(x) for x in v]


def _step_eager_and_graph(mesh, n, args, vt):
    from paper_2606_01598_amd.pme import Plan
    plan = Plan(mesh, 6, 0.30, max_atoms=n, keep_phi=True, concurrent=True)
    eager = plan.step(*args, *vt)
    plan.status()
    eager = {k: v.clone() for k, v in eager.items()}
    out = plan.step_capture(2, *args, *vt)
    plan.step_replay()
    plan.status()
    graph = {k: v.clone() for k, v in out.items()}
    return eager, graph


def _check(label, got, e_ref, per_atom_ref):
    e = host(got["energy"])
    e_rec = rel(e[0], e_ref[0])
    e_tot = rel(e.sum(), e_ref.sum())
    errs = {k: rms_rel(host(got[k]).reshape(len(per_atom_ref[k]), -1),
                       per_atom_ref[k].reshape(len(per_atom_ref[k]), -1)) for k in KEYS}
    print(label, f"E_recip {e_rec:.2e} E_lr {e_tot:.2e}",
          {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert e_rec <= E_REL_TOL and e_tot <= E_REL_TOL, (label, e_rec, e_tot)
    assert max(errs.values()) <= RMS_REL_TOL, (label, errs)


def test_step_32k_every_output():
    n, seed, mesh = 32000, 3, (100, 100, 100)
    print("case: pme_step 32k / 100^3, concurrent, eager + graph", flush=True)
    f, v, args, vt = _inputs(n, seed)
    eager, graph = _step_eager_and_graph(mesh, n, args, vt)
    for k in eager:
        assert torch.equal(eager[k], graph[k]), k
    ref = oracle_forward(f, mesh, 6, 0.30)
    hv = oracle_hvp(f, mesh, 6, 0.30, v)
    e_ref = np.array([ref.e_recip, ref.e_self_q, ref.e_self_mu])
    per_atom = {"dE_dpos": ref.dE_dpos, "dE_dq": ref.dE_dq, "dE_dmu": ref.dE_dmu,
                "g_pos": hv[0], "g_q": hv[1], "g_mu": hv[2]}
    _check("32k eager", eager, e_ref, per_atom)
    _check("32k graph", graph, e_ref, per_atom)


@pytest.mark.parametrize("name", ["128k", "1m"])
def test_step_sweep_sizes_sampled(name):
    n, seed, mesh, p, alpha = make_fullsize.WORKLOADS[name]
    print(f"case: pme_step {name} / {mesh[0]}^3, concurrent, eager + graph, sampled", flush=True)
    e_ref, idx, vals = make_fullsize.read(name)
    f, v, args, vt = _inputs(n, seed)
    eager, graph = _step_eager_and_graph(mesh, n, args, vt)
    for k in eager:
        assert torch.equal(eager[k], graph[k]), k
    per_atom = {k: vals[:, COLS[k]] for k in KEYS}
    ii = torch.tensor(idx, device=dev())
    for label, out in (("eager", eager), ("graph", graph)):
        got = {"energy": out["energy"], **{k: out[k][ii] for k in KEYS}}
        _check(f"{name} {label}", got, e_ref, per_atom)
