"""Lattice stencil layout of the finest operator (compact storage of regular regions).

Compiles tests/lattice_check.cpp with the library's host setup source and
runs it on level-0 operators of the native grid builder (16^3 plates k = 2,
16^3 thin sheet k = 2, 16^3 sphere k = 1 with a Dirichlet top) and of the
oracle (8^3 plates): every DOF appears once in the padded order, the tile
masks flag exactly the stencil rows, and an emulation of the stencil
kernel's addressing reproduces A x on those rows.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _assemble(desc):
    lv0 = desc["levels"][0]
    cp, cd, n = lv0["cell_ptr"], lv0["cell_dof"], lv0["n_dof"]
    rows, cols, vals = [], [], []
    for c in range(len(cp) - 1):
        ids = cd[cp[c]:cp[c + 1]]
        m = len(ids)
        K = desc["ke_val"][desc["ke_off"][c]:desc["ke_off"][c] + m * m].reshape(m, m)
        ok = ids >= 0
        I, J = np.meshgrid(ids, ids, indexing="ij")
        msk = ok[:, None] & ok[None, :]
        rows.append(I[msk])
        cols.append(J[msk])
        vals.append(K[msk])
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    # like the library: each entry sums its contributions in increasing
    # order of value, one after the other
    o = np.lexsort((v, c, r))
    r, c, v = r[o], c[o], v[o]
    start = np.flatnonzero(np.r_[True, (r[1:] != r[:-1]) | (c[1:] != c[:-1])])
    size = np.diff(np.r_[start, len(v)])
    acc = v[start].copy()
    for k in range(1, int(size.max())):
        m = size > k
        acc[m] += v[start[m] + k]
    K = sp.csr_matrix((acc, (r[start], c[start])), shape=(n, n))
    K.sort_indices()
    return K


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("lattice") / "lattice_check"
    src = [os.path.join(ROOT, "tests", "lattice_check.cpp"),
           os.path.join(ROOT, "paper_2607_17725_amd", "csrc", "setup_host.cpp")]
    subprocess.run([gxx, "-std=c++17", "-O2", "-fopenmp", "-o", str(exe)] + src, check=True)
    return exe


def _run(checker, tmp_path, K, lat, lat_n, want):
    files = []
    for name, arr in (("rp", K.indptr.astype(np.int64)), ("ci", K.indices.astype(np.int32)),
                      ("val", K.data.astype(np.float64)), ("lat", np.asarray(lat, dtype=np.int32))):
        f = tmp_path / name
        arr.tofile(f)
        files.append(str(f))
    out = subprocess.run([str(checker)] + files + [str(lat_n), str(want)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr


@pytest.mark.parametrize("name,N,k,want", [("c3", 16, None, 0.5), ("c4", 16, None, 0.3), ("c1", 16, None, 0.15)])
def test_native_grid_layout(name, N, k, want, checker, tmp_path):
    import synth
    from paper_2607_17725_amd import fvem
    w = synth.get_config(name, N=N, k=k)
    V, F = w.mesh()
    g = fvem.Grid(V, F, w.N, w.k, levels=w.levels, dirichlet_top=w.dirichlet_top)
    desc = g.describe()
    _run(checker, tmp_path, _assemble(desc), desc["levels"][0]["dof_lattice"], desc["levels"][0]["lattice_n"], want)


def test_oracle_layout(c3_small, checker, tmp_path):
    from oracle_desc import describe
    desc = describe(c3_small)
    _run(checker, tmp_path, _assemble(desc), desc["levels"][0]["dof_lattice"], desc["levels"][0]["lattice_n"], 0.05)
