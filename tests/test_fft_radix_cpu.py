"""Host check of the FFT radix stages the mesh passes run (csrc/fft_radix.h): the
in-register R-point DFTs (direct and split forms) and whole Stockham transforms
planned by radix_plan, the fused middle of the x pass (last forward stage, x g,
first inverse stage in registers), compiled for the host from the same header and
compared with a direct double-precision DFT (Eq. fft and its inverse); plus the
stage plans themselves (fewest stages, then the smallest largest radix)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("fftradix") / "check")
    subprocess.run([HIPCC, "--offload-host-only", "-x", "hip", "-std=c++17", "-O2",
                    os.path.join(HERE, "fft_radix_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return [line.split() for line in out.splitlines()]


def test_small_dfts_match_direct(report):
    rows = [r for r in report if r[0] == "dft"]
    assert {int(r[1]) for r in rows} == {2, 3, 4, 5, 6, 8, 10}
    for r in rows:
        assert float(r[3]) < 2e-6, r


def test_planned_transforms_match_direct(report):
    rows = [r for r in report if r[0] == "fft"]
    assert len(rows) == 2 * 18
    for r in rows:
        assert float(r[3]) < 1e-5, r


def test_fused_x_pass_matches_direct(report):
    """forward stages, last forward stage x g x first inverse stage in registers, the
    reversed plan's remaining stages == IDFT(g DFT(x)), unnormalised"""
    rows = [r for r in report if r[0] == "fused"]
    assert len(rows) == 17
    for r in rows:
        assert float(r[2]) < 2e-5, r


def test_stage_plans(report):
    plans = {int(r[1]): [int(x) for x in r[2].split(",")] if len(r) > 2 else []
             for r in report if r[0] == "plan"}
    assert plans[100] == [10, 10]
    assert plans[64] == [8, 8]
    assert plans[160] == [8, 5, 4]
    assert plans[320] == [8, 8, 5]
    assert plans[1] == []
    for n, rs in plans.items():
        prod = 1
        for x in rs:
            prod *= x
        assert prod == n
    noplan = {int(r[1]) for r in report if r[0] == "noplan"}
    assert noplan == {7, 14, 22, 49}
