"""Build the oracle's C library (``oracle/_gemm_f64.so``) with gcc.

TEST INFRASTRUCTURE ONLY: the product library never links or loads it.

Flags: ``-ffp-contract=off`` and no ``-ffast-math`` so that every product and
every sum of the reference loop is rounded separately to binary64, in the
order the source states.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gemm_f64.c")
LIB = os.path.join(HERE, "_gemm_f64.so")

CFLAGS = ["-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-std=c11", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
