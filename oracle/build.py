"""Compile the oracle (plain C, FP64, one thread) into oracle/liboracle.so.

Test infrastructure only.  Built with -O2 and without floating-point
contraction or fast-math so that every expression is evaluated as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "vx_oracle.c")]


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB + ".tmp"] + SRC + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built():
    newest = max(os.path.getmtime(p) for p in SRC + [os.path.join(HERE, "vx_oracle.h")])
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
