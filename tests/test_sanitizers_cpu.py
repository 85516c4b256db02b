"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The host BVH builder (paper_2305_04403_amd/csrc/bvh_build.cpp) with a
  structural checker over random and degenerate box sets
  (tests/sanitize/bvh_check.cpp), built with g++ and both sanitizers.
* The oracle's C sources built with both sanitizers (oracle/build.py,
  sanitize=True), every entry point exercised on tiny inputs
  (tests/sanitize/oracle_exercise.py) in a child process that preloads the
  sanitizer runtimes; any finding aborts the child.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


pytestmark = pytest.mark.skipif(shutil.which("g++") is None or _runtime("libasan.so") is None,
                                reason="no g++ with the sanitizer runtimes")


def test_bvh_builder_under_sanitizers(tmp_path):
    exe = tmp_path / "bvh_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "tests", "sanitize", "bvh_check.cpp"),
                    os.path.join(ROOT, "paper_2305_04403_amd", "csrc", "bvh_build.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_oracle_under_sanitizers():
    from oracle import build
    lib = build.build(sanitize=True)
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = ":".join(p for p in (_runtime("libasan.so"), _runtime("libubsan.so")) if p)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize", "oracle_exercise.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
