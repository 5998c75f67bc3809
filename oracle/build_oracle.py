"""Compile the FP64 CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain C, gcc, -O2 with floating-point contraction disabled so that every
multiply and add rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nplbm_oracle.c")
SRC3 = os.path.join(HERE, "nplbm_oracle3d.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function", SRC, SRC3, "-o", tmp,
           "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
