"""Build the FP64 oracle shared library (test infrastructure only).

Plain `gcc -O2` with OpenMP for threading over points; no fast-math, so every
operation is IEEE double precision as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
# the same sources under AddressSanitizer and UndefinedBehaviorSanitizer
# (any finding aborts); loaded by a process that preloads the two runtimes
LIB_SANITIZED = os.path.join(HERE, "liboracle_sanitized.so")
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SANITIZED if sanitize else LIB
    flags = ["-O1"] + SANITIZE_FLAGS if sanitize else ["-O2"]
    # written under a name of this process and renamed into place, so that a
    # process loading the library (parallel test workers) never sees it half
    # written
    tmp = f"{out}.{os.getpid()}.tmp"
    cmd = ["gcc", "-std=c11", *flags, "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, os.path.join(HERE, "oracle.c"), os.path.join(HERE, "mlp.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    try:
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
