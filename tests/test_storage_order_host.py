"""The level-major chunk order of stored diagonals, checked on the host: the
library's position function (storage_order.h, built with hipcc as host code)
is a permutation of each diagonal's N - |d| entries, keeps row pairs
adjacent, is the identity in natural order, and gives every strided tile's
window one contiguous stretch per chunk column (tests/c/storage_order_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_storage_order_positions(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "storage_order_check")
    cmd = [hipcc, "-x", "hip", "-O2", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(ROOT, "tests", "c", "storage_order_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-2000:]
    assert "cases checked" in run.stdout
