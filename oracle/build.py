"""Compile the oracle's C code into oracle/liboracle.so with gcc.

Test infrastructure: the flags keep every floating-point operation separate
and correctly rounded (-ffp-contract=off, no fast-math); OpenMP runs the
colour-parallel CPU baseline loop on all host cores.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["flux_oracle.c", "hex_oracle.c", "step_oracle.c", "cpu_parallel.c"]
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", OUT + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
