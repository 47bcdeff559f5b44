"""Build step for the CPU oracle's C library (test infrastructure only).

Compiles ``oracle.c`` into ``liboracle.so`` beside it with gcc, at -O2 with
floating-point contraction off and no fast-math, so every floating-point
operation in the oracle is exactly the one its source writes.  OpenMP is
enabled for the multi-threaded full-grid forms (threads split rows or
planes; the per-element arithmetic is that of the sequential routines).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-Wall", "-fopenmp"]


def build(force=True):
    """Compile liboracle.so; returns its path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
