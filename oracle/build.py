"""Build the oracle's C library (liboracle.so) with gcc.

TEST INFRASTRUCTURE: the oracle is only ever loaded by the test suite, the
smoke check and the benchmark's CPU-baseline leg.  Plain -O2 (no fast-math,
no FMA contraction on the default x86-64 target) so the FP64 arithmetic is
the IEEE evaluation of the written expressions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-ffp-contract=off", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
