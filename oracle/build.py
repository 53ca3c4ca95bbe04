"""Compile the oracle's C grid operators (test infrastructure only).

gcc -O2 -fopenmp, deliberately without -ffast-math (Section 2.2 warns that
aggressive optimisation can spoil the scaling invariance of the Cholesky
step).  The result, ``_grid_ops.so``, sits beside its source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "grid_ops.c")
LIB = os.path.join(HERE, "_grid_ops.so")


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
