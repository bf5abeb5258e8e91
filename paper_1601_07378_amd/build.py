"""Build libvloc.so in-tree with hipcc for gfx950.

All device code is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``) and with
``-fno-signed-zeros`` so that additions of known zeros fold away.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libvloc.so")
SOURCES = ["kernels.hip", "reduce.hip", "plan.cpp", "api.cpp"]
ARCH = os.environ.get("VLOC_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    out = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-fno-signed-zeros",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", out]
    # the .cpp files call the HIP runtime, so every source is compiled as HIP
    cmd += ["-x", "hip"] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libvloc.so")
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
