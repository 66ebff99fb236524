"""Host C++ under the address and undefined-behaviour sanitizers.

The library's host setup routines (sliced storage, level order, Galerkin
products, lattice layout) and the native grid builder (cut cells,
hierarchy, VEM operators, prolongation) are compiled with g++ and
-fsanitize=address,undefined (no HIP code is involved) and run on small
inputs: the setup checks, the lattice-layout check on a builder operator,
and the builder on the 8^3 plates (k = 2) and the 8^3 thin sheet (k = 2).
Any sanitizer report fails the test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_17725_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _gxx():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    return gxx


def _build(tmp_path, name, sources):
    exe = tmp_path / name
    subprocess.run([_gxx(), "-std=c++17", "-O1", "-g", "-fopenmp"] + SAN + ["-o", str(exe)] + sources, check=True)
    return exe


def _run(args):
    out = subprocess.run([str(a) for a in args], capture_output=True, text=True, env=ENV, timeout=600)
    print(out.stdout[-2000:])
    assert out.returncode == 0 and "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, \
        out.stdout[-2000:] + out.stderr[-4000:]


def test_setup_routines_sanitized(tmp_path):
    exe = _build(tmp_path, "host_setup_check",
                 [os.path.join(ROOT, "tests", "host_setup_check.cpp"), os.path.join(CSRC, "setup_host.cpp")])
    _run([exe])


@pytest.mark.parametrize("name", ["c3", "c4"])
def test_native_builder_sanitized(name, tmp_path):
    import synth
    exe = _build(tmp_path, "builder_check",
                 [os.path.join(ROOT, "tests", "builder_check.cpp")] +
                 [os.path.join(CSRC, f) for f in ("grid.cpp", "vem.cpp", "geom.cpp")])
    w = synth.get_config(name, N=8)
    V, F = w.mesh()
    np.ascontiguousarray(V, dtype=np.float64).tofile(tmp_path / "V")
    np.ascontiguousarray(F, dtype=np.int32).tofile(tmp_path / "F")
    _run([exe, tmp_path / "V", tmp_path / "F", w.N, w.k, w.levels])
