"""The lattice stencil layout of the finest operator on the GPU.

Native-grid problems at 16^3 (plates and thin sheet, k = 2; sphere with a
Dirichlet top, k = 1) are built twice from one description: with the
lattice stencil layout forced on and with every row in sliced storage.
Both must apply the same K, give the same V-cycles and converge to the same
pressure, which must equal a sparse direct solve of K assembled on the host
from the same element blocks.  The 128^3 plates (the benchmark workload)
use the layout by default; their stencil share is checked here too.
"""
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_lattice_layout import _assemble   # noqa: E402

_CACHE = {}


def _pair(name, N):
    import synth
    from paper_2607_17725_amd import fvem
    if (name, N) not in _CACHE:
        w = synth.get_config(name, N=N)
        V, F = w.mesh()
        print(f"[gpu stencil] building {name}@{N}", flush=True)
        g = fvem.Grid(V, F, w.N, w.k, levels=w.levels, dirichlet_top=w.dirichlet_top)
        desc = g.describe()
        on = fvem.Hierarchy(desc, lattice_min_fraction=1e-6)
        off = fvem.Hierarchy(desc, lattice_min_fraction=-1.0)
        _CACHE[(name, N)] = (w, g, desc, on, off)
    return _CACHE[(name, N)]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


CASES = [("c3", 16), ("c4", 16), ("c1", 16)]


@pytest.mark.parametrize("name,N", CASES)
def test_stencil_layout_applies_K(name, N):
    from paper_2607_17725_amd import fvem
    w, g, desc, on, off = _pair(name, N)
    st = on.level_stencil(0)
    print(f"[gpu stencil] {name}@{N}: {st}", flush=True)
    assert st["rows"] > 0 and off.level_stencil(0)["rows"] == 0
    K = _assemble(desc)
    x = np.random.default_rng(3).standard_normal(on.n_dof)
    ref = K @ x
    scale = abs(K) @ np.abs(x)
    for h in (on, off):
        y = h.apply(fvem.OP_K, _dev(x)).cpu().numpy()
        assert np.max(np.abs(y - ref) / scale) < 1e-14
    # the read-back operator (stencil rows rebuilt from the class tables)
    rp, ci, va = on.level_matrix(0)
    Kr = sp.csr_matrix((va, ci, rp), shape=K.shape)
    assert abs(Kr - K).max() <= 1e-15 * abs(K).max()
    # every coarser level: the layout chosen per level holds the same
    # operator as sliced storage, value for value
    for l in range(1, on.n_levels):
        n = on.level_rows(l)
        rp, ci, va = on.level_matrix(l)
        A_on = sp.csr_matrix((va, ci, rp), shape=(n, n))
        rp, ci, va = off.level_matrix(l)
        A_off = sp.csr_matrix((va, ci, rp), shape=(n, n))
        print(f"[gpu stencil] {name}@{N} level {l}: {on.level_stencil(l)}", flush=True)
        assert off.level_stencil(l)["rows"] == 0
        assert abs(A_on - A_off).max() == 0.0


@pytest.mark.parametrize("name,N", CASES)
def test_stencil_layout_vcycle_and_solve(name, N):
    from paper_2607_17725_amd import fvem
    import synth
    w, g, desc, on, off = _pair(name, N)
    n = on.n_dof
    r = np.random.default_rng(4).standard_normal(n)
    r = _dev(on.apply(fvem.OP_PROJECT, _dev(r)).cpu().numpy())
    # the bars of the oracle V-cycle parity: the two layouts sum rows in
    # different orders, and the shifted coarsest solve amplifies that rounding
    for op, tol in ((fvem.OP_VCYCLE, 1e-8), (fvem.OP_VCYCLE32, 1e-4)):
        z1 = on.apply(op, r).cpu().numpy()
        z2 = off.apply(op, r).cpu().numpy()
        assert np.linalg.norm(z1 - z2) <= tol * np.linalg.norm(z2)
    K = _assemble(desc)
    u = (synth.normal_field(g.vertices, 0) if w.field_kind == "normal" else synth.fourier_field(g.vertices, 0)).ravel()
    b = on.apply(fvem.OP_B, _dev(u)).cpu().numpy()
    comp = desc["component"]
    if (comp >= 0).any():
        # pure Neumann: pin one DOF of the component and re-centre
        keep = np.arange(1, n)
        p_ref = np.zeros(n)
        p_ref[keep] = spl.splu(K[keep][:, keep].tocsc()).solve(b[keep])
        p_ref -= p_ref.mean()
    else:
        p_ref = spl.splu(K.tocsc()).solve(b)
    its = []
    for h in (on, off):
        for prec in (fvem.PREC_FP64, fvem.PREC_MIXED):
            p, st = h.solve(_dev(u), tol=1e-10, precision=prec)
            p = p.cpu().numpy()
            res = np.linalg.norm(b - K @ p) / np.linalg.norm(b)
            assert res <= 1.01e-10
            assert np.linalg.norm(p - p_ref) <= 1e-7 * np.linalg.norm(p_ref)
            its.append(st["iterations"])
    print(f"[gpu stencil] {name}@{N} iterations (stencil fp64, mixed; sliced fp64, mixed): {its}", flush=True)
