"""Build the FP64 oracle shared library (test infrastructure only).

Plain `gcc -O2` with OpenMP for threading over points; no fast-math, so every
operation is IEEE double precision as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB, os.path.join(HERE, "oracle.c"), os.path.join(HERE, "mlp.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
