"""Host-side setup routines of the library against dense brute force.

Compiles tests/host_setup_check.cpp together with the library's pure C++
setup source (no HIP) and runs it: sliced storage round trip (ragged last
slice, empty rows), the level order, symmetric renumbering and its inverse,
transpose, block assembly, the element-wise Galerkin product P^T A P and the
scaled Gershgorin bound.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_setup_routines(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "host_setup_check"
    src = [os.path.join(ROOT, "tests", "host_setup_check.cpp"),
           os.path.join(ROOT, "paper_2607_17725_amd", "csrc", "setup_host.cpp")]
    subprocess.run([gxx, "-std=c++17", "-O1", "-fopenmp", "-o", str(exe)] + src, check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
