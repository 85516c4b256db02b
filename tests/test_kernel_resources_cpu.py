"""Register budgets of the hot kernels (CPU: hipcc reports each kernel's
resource usage at compile time for gfx950).  The walk is latency-bound, so a
change that costs a wave per SIMD costs a fifth of the throughput or more;
these bounds keep the occupancy each kernel is measured at."""
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, mangled-name prefix, description, VGPR bound, waves per SIMD)
BUDGETS = [
    ("wob.hip", "_ZN3wob11walk_kernelIfLi3ELi3ELb0ELb0ELi64ELi0EE", "single layer, 3D FP32 solve (two points pooled per lane group)", 128, 4),
    ("wob.hip", "_ZN3wob11walk_kernelIfLi3ELi1ELb0ELb0ELi64ELi0EE", "double layer, 3D FP32 solve", 96, 5),
    ("wob.hip", "_ZN3wob11walk_kernelIfLi3ELi1ELb0ELb0ELi64ELi2EE", "double layer gradient (with the split)", 128, 4),
    ("wob.hip", "_ZN3wob11walk_kernelIfLi3ELi3ELb0ELb0ELi64ELi1EE", "single layer, control variate", 128, 4),
    ("batch.hip", "_ZN3wob12batch_kernelIfLi3ELi64ELi0EE", "batched, every form, 64 lanes", 128, 4),
]


def _remarks(src):
    cmd = [HIPCC, "-c", "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
           os.path.join(ROOT, "paper_2305_04403_amd", "csrc", src), "-o", os.devnull]
    return subprocess.run(cmd, capture_output=True, text=True, timeout=900).stderr


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_hot_kernels_keep_their_register_budgets():
    with ThreadPoolExecutor(2) as ex:
        text = dict(zip(("wob.hip", "batch.hip"), ex.map(_remarks, ("wob.hip", "batch.hip"))))
    for src, name, what, bound, waves in BUDGETS:
        m = re.search(re.escape(name) + r".*?VGPRs: (\d+).*?Occupancy \[waves/SIMD\]: (\d+)", text[src], re.S)
        assert m, f"{what}: no resource remark for {name}"
        vgprs, occ = int(m.group(1)), int(m.group(2))
        assert vgprs <= bound and occ >= waves, f"{what}: {vgprs} VGPRs, {occ} waves per SIMD"
