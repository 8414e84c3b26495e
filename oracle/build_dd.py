"""Build the oracle's double-double GEMM helper (oracle/libddgemm.so) with gcc.

TEST INFRASTRUCTURE ONLY. Called from the repository's build step and, when the
shared object is missing, lazily by oracle.dd.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dd_gemm.c")
LIB = os.path.join(HERE, "libddgemm.so")

# -mfma: hardware fused multiply-add for TwoProd (every x86-64 host from the
# last decade has it); -ffp-contract=off keeps a*b separate from the fma that
# measures its rounding error; no fast-math anywhere.
CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-mfma", "-ffp-contract=off",
          "-fno-fast-math", "-std=c99"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
