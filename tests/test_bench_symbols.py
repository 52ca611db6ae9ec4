"""bench.py's profiler names against the kernels in the library sources (no GPU).

bench.py matches rocprofv3's per-kernel statistics to its launch-timer kinds by the
names the profiler prints (a template kernel prints every template argument,
defaults included).  These checks keep its tables in step with the sources: every
name it uses is a __global__ kernel of csrc, with as many template arguments as
the kernel has parameters and of their kinds; the slab test it uses to name the
transform kernels agrees with the library's own constant; and the workload meshes
take the layouts the committed kernel statistics show."""
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_01598_amd", "csrc")


def _skip_group(text, i):
    """Index just past the balanced parenthesis group that starts at text[i]."""
    assert text[i] == "("
    depth = 0
    for j in range(i, len(text)):
        if text[j] == "(":
            depth += 1
        elif text[j] == ")":
            depth -= 1
            if depth == 0:
                return j + 1
    raise ValueError("unbalanced parentheses")


def _kernels():
    """name -> list of template parameter kinds ('int', 'bool'); [] if not a template."""
    out = {}
    for fn in sorted(os.listdir(CSRC)):
        if not fn.endswith(".hip"):
            continue
        text = open(os.path.join(CSRC, fn)).read()
        for m in re.finditer(r"__global__\s+void\b", text):
            i = m.end()
            while True:
                while text[i].isspace():
                    i += 1
                w = re.match(r"(__launch_bounds__|__attribute__)\s*", text[i:])
                if not w:
                    break
                i = _skip_group(text, i + w.end())
            name = re.match(r"\w+", text[i:]).group(0)
            head = text[:m.start()].rstrip()
            params = []
            t = re.search(r"template\s*<([^<>]*)>$", head)
            if t:
                for p in t.group(1).split(","):
                    params.append(p.split()[0])
            if name in out:
                assert out[name] == params, name
            out[name] = params
    return out


def _names():
    names = set(bench.KERNEL_SYMBOL.values()) | set(bench.FUSED_SYMBOL.values())
    names |= set(bench.BAND_SYMBOL.values())
    names |= {bench.FUSED_STEP_SPREAD, bench.BAND_STEP_SPREAD}
    for s in bench.PENCIL_SYMBOL.values():
        names |= set(s.split("+"))
    for kind in bench.KERNEL_SYMBOL:
        for step in (False, True):
            for fused, band in ((False, False), (True, False), (False, True)):
                for slab in (True, False):
                    names |= set(bench.kernel_symbol(kind, step, fused, band, slab).split("+"))
    return sorted(names)


@pytest.mark.parametrize("symbol", _names())
def test_profiler_name_is_a_kernel_of_the_sources(symbol):
    kernels = _kernels()
    m = re.fullmatch(r"(\w+)(?:<(.*)>)?", symbol)
    assert m, symbol
    name, args = m.group(1), m.group(2)
    assert name in kernels, f"{name} is not a __global__ kernel in csrc"
    params = kernels[name]
    got = [a.strip() for a in args.split(",")] if args is not None else []
    assert len(got) == len(params), (symbol, params)
    for a, kind in zip(got, params):
        if kind == "bool":
            assert a in ("true", "false"), symbol
        else:
            assert re.fullmatch(r"-?\d+", a), symbol


def test_step_spread_names_take_the_tangent_records():
    # under pme_step the forward plane spread reads the tangent records (last
    # template argument true); the separate forward spreads do not
    assert bench.kernel_symbol("spread", True, fused=True) == bench.FUSED_STEP_SPREAD
    assert bench.kernel_symbol("spread", True, band=True) == bench.BAND_STEP_SPREAD
    assert bench.FUSED_STEP_SPREAD.endswith(", true>")
    assert bench.BAND_STEP_SPREAD.endswith(", true>")
    for s in list(bench.FUSED_SYMBOL.values()) + list(bench.BAND_SYMBOL.values()):
        assert s.endswith(", false>"), s
    assert bench.kernel_symbol("gather_hvp", True) == "k_gather_hvp<6, true>"
    assert bench.kernel_symbol("gather_hvp", False) == "k_gather_hvp<6, false>"


def test_slab_limit_matches_the_library():
    text = open(os.path.join(CSRC, "kernels.h")).read()
    m = re.search(r"constexpr int kSlabLdsMax = ([^;]+);", text)
    assert m
    assert eval(m.group(1), {"__builtins__": {}}) == bench.SLAB_LDS_MAX


@pytest.mark.parametrize("mesh,slab", [((64, 64, 64), True), ((100, 100, 100), True),
                                       ((160, 160, 160), False), ((320, 320, 320), False)])
def test_workload_mesh_layouts(mesh, slab):
    # the 32k kernel statistics show k_slab_inv on 100^3; those of 128k and 1M show
    # the pencil passes (k_ffty) on 160^3 and 320^3
    assert bench.is_slab(mesh) == slab
