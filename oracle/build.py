"""Compile the CPU oracle (plain C, FP64) into ``oracle/_build/liboracle.so``.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU baseline
load the result.  Run as ``python oracle/build.py``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mg_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
OUT = os.path.join(OUT_DIR, "liboracle.so")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = OUT + ".tmp"
    # -O3 without fast-math and without contraction: IEEE FP64 semantics, no reassociation of
    # the plain loops and no fused multiply-adds, so every optimisation level gives the same
    # bits.  x86-64-v3 (AVX2) rather than -march=native: the library may run on another host
    # than the one that built it.
    cmd = ["gcc", "-std=c11", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
