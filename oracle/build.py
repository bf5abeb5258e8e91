"""Build step for the CPU oracle library (test infrastructure only).

Compiles ``vloc_oracle.c`` with gcc into ``liboracle_vloc.so`` next to this
file.  Plain C, FP64, OpenMP over bands.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vloc_oracle.c")
LIB = os.path.join(HERE, "liboracle_vloc.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
