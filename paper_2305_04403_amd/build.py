"""Build libwob.so (HIP, gfx950) in-tree.

    python -m paper_2305_04403_amd.build

hipcc compiles the kernels for gfx950 only.  Packed-FP32 instruction
selection is disabled (-packed-fp32-ops): ordinary scalar FP32 code is
emitted for every float operation.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwob.so")
ARCH = os.environ.get("WOB_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    cmds, objs = [], []
    for src in ("wob.hip", "order.hip", "batch.hip", "mlp.hip", "forward.hip", "probe.hip"):
        obj = os.path.join(obj_dir, src.replace(".hip", ".o"))
        cmds.append([hipcc, "-c", *HIP_FLAGS, os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in ("bvh_build.cpp",):
        obj = os.path.join(obj_dir, src.replace(".cpp", ".o"))
        cmds.append(["g++", "-c", "-O2", "-std=c++17", "-fPIC", "-Wall", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the translation units are independent: compile them side by side
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for f in [pool.submit(subprocess.check_call, cmd) for cmd in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
