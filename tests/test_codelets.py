"""The register DFT codelets of the transform kernels (csrc/dft_codelets.h)
against the DFT definition, on the host: every size a plan may use, both
signs, FP64 and FP32.  Built with hipcc as host code only; no device."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1601_07378_amd", "csrc")


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("codelets")
    exe = str(d / "codelet_check")
    src = os.path.join(ROOT, "tests", "codelet_check.cpp")
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", "-I", CSRC, src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = {}
    for line in out.strip().splitlines():
        r, *errs = line.split()
        rows[int(r)] = [float(e) for e in errs]
    return rows


SIZES = [1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32]


def test_every_codelet_size(results):
    assert sorted(results) == SIZES


@pytest.mark.parametrize("R", SIZES)
def test_codelet_matches_dft(results, R):
    d_minus, d_plus, f_minus, f_plus = results[R]
    assert d_minus <= 1e-15 and d_plus <= 1e-15, (R, d_minus, d_plus)
    assert f_minus <= 4e-7 and f_plus <= 4e-7, (R, f_minus, f_plus)
