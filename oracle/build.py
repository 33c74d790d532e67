"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libpsvd_oracle.so.

Plain gcc, OpenMP, no BLAS/LAPACK.  `-ffp-contract=off` keeps every product
and sum as written (no fused multiply-add contraction).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psvd_oracle.c")
LIB = os.path.join(HERE, "libpsvd_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O3", "-mavx2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
        "-std=c11", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
