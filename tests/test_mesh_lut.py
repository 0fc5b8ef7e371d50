"""The mesh look-up table that the vertex kernels use to bracket a frequency
(build_mesh_lut and bracket_lut in csrc/device_common.h), compiled for the
host and checked against a plain binary search: same bracket indices and
bitwise the same interpolation weights on logarithmic, linear, clustered and
random meshes of 2 to 128 points, at every mesh point and its floating-point
neighbours, every bucket boundary, midpoints and random arguments; a NaN
argument stays in bounds.  Host code only (no GPU)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not found")


def test_mesh_lut_matches_binary_search(tmp_path):
    exe = tmp_path / "mesh_lut_check"
    src = os.path.join(ROOT, "tests", "mesh_lut_check.cpp")
    subprocess.run([_hipcc(), "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2109_13317_amd", "csrc"), src, "-o", str(exe)],
                   check=True, capture_output=True, text=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().splitlines()[-1].startswith("ok:")
