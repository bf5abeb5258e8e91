"""The host planner and the C oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc/g++, host code only) and run on the
geometries and error paths the other tests use."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1601_07378_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g", "-O1"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-3000:]
    return res.stdout


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("gcc/g++ not available")
    return tmp_path_factory.mktemp("sanitize")


def test_planner_under_sanitizers(tmp):
    exe = str(tmp / "planner")
    _run(["g++", "-std=c++17"] + SAN + ["-I", CSRC, "-I", os.path.join(ROOT, "include"),
                                        os.path.join(ROOT, "tests", "sanitize_planner.cpp"),
                                        os.path.join(CSRC, "plan.cpp"), "-o", exe])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert out.strip().endswith("OK"), out


def test_oracle_under_sanitizers(tmp):
    exe = str(tmp / "oracle")
    _run(["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "tests", "sanitize_oracle.c"),
                                      os.path.join(ROOT, "oracle", "vloc_oracle.c"), "-o", exe,
                                      "-lm"])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert out.strip().endswith("OK"), out
