"""Build libvloc.so in-tree with hipcc for gfx950.

All device code is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``) and with
``-fno-signed-zeros`` so that additions of known zeros fold away.  Sources
compile to objects in parallel (the transform kernels once per precision and
launcher part)
and are linked into one shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libvloc.so")
OBJDIR = os.path.join(PKG, "_build")
ARCH = os.environ.get("VLOC_OFFLOAD_ARCH", "gfx950")
# (source, object, extra defines)
UNITS = [
    ("kernels.hip", f"kernels_{prec}_{part}.o", [f"-DVLOC_ONLY_{prec.upper()}",
                                                 f"-DVLOC_PART_{part.upper()}"])
    for prec in ("f64", "f32") for part in ("full_apply", "full_aux", "rows", "stick")
] + [
    ("kernels.hip", f"kernels_{prec}_tune{gi}.o",
     [f"-DVLOC_ONLY_{prec.upper()}", "-DVLOC_PART_TUNE", f"-DVLOC_TUNE_T={t}",
      f"-DVLOC_TUNE_G={gi}"])
    for prec, t in (("f64", "double"), ("f32", "float")) for gi in range(3)
] + [
    ("reduce.hip", "reduce.o", []),
    ("plan.cpp", "plan.o", []),
    ("api.cpp", "api.o", []),
]
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fno-signed-zeros",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for src, obj, defs in UNITS:
        # the .cpp files call the HIP runtime, so every source is compiled as HIP
        jobs.append(["hipcc"] + FLAGS + defs + ["-c", "-x", "hip", os.path.join(CSRC, src),
                                               "-o", os.path.join(OBJDIR, obj)])
    workers = min(len(jobs), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_run, j, verbose) for j in jobs]:
            f.result()
    out = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] +
         [os.path.join(OBJDIR, o) for _, o, _ in UNITS], verbose)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
