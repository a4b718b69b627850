"""Tile shapes shared by the launch planner and the kernels, checked on the
host (tests/c/tile_shapes_check.cpp, plain C++ built with g++): every
(dtype, batch, closed/open) shape gives each tile row a thread and fits its
LDS budget; 5 complex64 states take 4096-row tiles in the whole 160 KiB of
a CU's LDS (2048 rows under a 128 KiB device limit); 2 complex128 states
take 4096-row tiles."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tile_shapes(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tile_shapes_check")
    cmd = [gxx, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "tile_shapes_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-2000:]
    assert "32 shapes checked" in run.stdout
