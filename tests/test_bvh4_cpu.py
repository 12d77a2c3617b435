"""The four-wide BVH of the dense-scene kernel build, checked on the host:
tests/cpp/bvh4_check.cpp builds seeded scenes host-only through the C ABI and
emulates the kernel's quantized slab tests in float32 against exact AABB
hits (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_2012_10357_amd")


def test_four_wide_bvh_reaches_every_hit(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(os.path.join(LIB_DIR, "libprocray.so")):
        pytest.fail("libprocray.so is missing: run __graft_entry__.build() first")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "bvh4_check")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(LIB_DIR, "csrc"), os.path.join(ROOT, "tests", "cpp", "bvh4_check.cpp"),
           "-o", exe, "-L", LIB_DIR, "-lprocray", "-Wl,-rpath," + LIB_DIR]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert "missed hits 0" in r.stdout
