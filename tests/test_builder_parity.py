"""Parity of the native grid builder (host C++) with the oracle, entry by entry.

Both sides build the cut-cell grid, VEM operators and hierarchy from the same
boundary mesh with independent code (different quadratures and monomial
frames).  DOFs are matched by (kind, support point); the matrices must then
agree entry by entry:
* the hierarchy shape (cells and DOFs per level, prolongation nonzeros) exactly;
* K, B, every P_l and the velocity-correction operators (Pi_1, grad Pi_k,
  cell mass, vertex average) to 1e-10 relative per row; 1e-6 for the 1e-5-thin sheet,
  whose sliver cells (aspect ratio ~1e3) amplify the ~1e-16 differences of
  the two sides' vertex coordinates through ill-conditioned local systems.
No GPU is needed: the builder is host code.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.spatial import cKDTree

from conftest import oracle_problem


def _native(name, N):
    import synth
    from paper_2607_17725_amd import fvem
    import os
    if not os.path.exists(fvem.LIB_PATH):
        pytest.skip("libfvem.so not built")
    w = synth.get_config(name, N=N)
    V, F = w.mesh()
    return fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top)


def _match(p_nat, k_nat, p_ora, k_ora):
    """perm[i] = oracle index of native DOF i."""
    assert len(p_nat) == len(p_ora)
    perm = np.full(len(p_nat), -1)
    for kind in range(4):
        a = np.nonzero(k_nat == kind)[0]
        b = np.nonzero(k_ora == kind)[0]
        assert len(a) == len(b), f"kind {kind}: {len(a)} vs {len(b)}"
        if len(a) == 0:
            continue
        d, j = cKDTree(p_ora[b]).query(p_nat[a])
        assert d.max() < 1e-9, f"kind {kind}: unmatched support point ({d.max()})"
        perm[a] = b[j]
    assert len(set(perm.tolist())) == len(perm)
    return perm


def _assemble(desc, n):
    lv = desc["levels"][0]
    rows, cols, vals = [], [], []
    for c in range(len(lv["cell_ptr"]) - 1):
        d = lv["cell_dof"][lv["cell_ptr"][c]:lv["cell_ptr"][c + 1]]
        m = len(d)
        K = desc["ke_val"][desc["ke_off"][c]:desc["ke_off"][c] + m * m].reshape(m, m)
        keep = d >= 0
        rows.append(np.repeat(d[keep], keep.sum()))
        cols.append(np.tile(d[keep], keep.sum()))
        vals.append(K[np.ix_(keep, keep)].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def _assemble_B(desc, n):
    lv = desc["levels"][0]
    rows, cols, vals = [], [], []
    for c in range(len(lv["cell_ptr"]) - 1):
        d = lv["cell_dof"][lv["cell_ptr"][c]:lv["cell_ptr"][c + 1]]
        verts = desc["cell_vert"][desc["cell_vptr"][c]:desc["cell_vptr"][c + 1]]
        m, nv = len(d), len(verts)
        Bm = desc["be_val"][desc["be_off"][c]:desc["be_off"][c] + m * 3 * nv].reshape(m, 3 * nv)
        vc = (3 * verts[:, None] + np.arange(3)[None, :]).ravel()
        keep = d >= 0
        rows.append(np.repeat(d[keep], len(vc)))
        cols.append(np.tile(vc, keep.sum()))
        vals.append(Bm[keep].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, 3 * desc["n_vert"]))


def _rel_rows(A, B):
    """max over rows of |A - B|_inf / |B|_row,inf."""
    D = abs(A - B).tocsr()
    scale = np.asarray(abs(B).max(axis=1).todense()).ravel()
    # rows that nearly cancel (entries far below the matrix scale) are
    # compared against a floor of 1e-4 of the matrix scale
    scale = np.maximum(scale, 1e-4 * scale.max())
    return float((np.asarray(D.max(axis=1).todense()).ravel() / scale).max())


def _velocity_ops(desc, n):
    """Pi, G, M, Av of the cell-field velocity correction, assembled from the description's blocks."""
    lv = desc["levels"][0]
    nc = len(lv["cell_ptr"]) - 1
    nv = desc["n_vert"]
    X = desc["vert_xyz"].reshape(-1, 3)
    geom = desc["cell_geom"].reshape(-1, 5)
    W = np.zeros(nv)
    for c in range(nc):
        W[desc["cell_vert"][desc["cell_vptr"][c]:desc["cell_vptr"][c + 1]]] += geom[c, 4]
    T = {k: ([], [], []) for k in ("Pi", "G", "M", "Av")}
    for c in range(nc):
        d = lv["cell_dof"][lv["cell_ptr"][c]:lv["cell_ptr"][c + 1]]
        verts = desc["cell_vert"][desc["cell_vptr"][c]:desc["cell_vptr"][c + 1]]
        m, nvE = len(d), len(verts)
        blk = desc["vc_val"][desc["vc_off"][c]:desc["vc_off"][c] + 4 * nvE + 12 * m + 16]
        pi1 = blk[:4 * nvE].reshape(4, nvE)
        gk = blk[4 * nvE:4 * nvE + 12 * m].reshape(3, 4, m)
        m1 = blk[4 * nvE + 12 * m:].reshape(4, 4)
        z = np.concatenate([np.ones((nvE, 1)), (X[verts] - geom[c, :3]) / geom[c, 3]], axis=1)
        keep = d >= 0
        for comp in range(3):
            rows = 12 * c + 4 * comp + np.arange(4)
            for key, r, cc, v in (
                    ("Pi", np.repeat(rows, nvE), np.tile(3 * verts + comp, 4), pi1.ravel()),
                    ("G", np.repeat(rows, keep.sum()), np.tile(d[keep], 4), gk[comp][:, keep].ravel()),
                    ("M", np.repeat(rows, 4), np.tile(rows, 4), m1.ravel()),
                    ("Av", np.repeat(3 * verts + comp, 4), np.tile(rows, nvE),
                     ((geom[c, 4] / W[verts])[:, None] * z).ravel())):
                T[key][0].append(r)
                T[key][1].append(cc)
                T[key][2].append(v)
    shapes = {"Pi": (12 * nc, 3 * nv), "G": (12 * nc, n), "M": (12 * nc, 12 * nc), "Av": (3 * nv, 12 * nc)}
    return {k: sp.csr_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))), shape=shapes[k])
            for k, (r, c, v) in T.items()}


TOL = {"c1": 1e-10, "c2": 1e-10, "c3": 1e-10, "c4": 1e-6}


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4"])
def test_native_builder_matches_oracle(name):
    tol = TOL[name]
    pb = oracle_problem(name, 8)
    g = _native(name, 8)
    desc = g.describe()
    L = len(pb.meshes)
    assert len(desc["levels"]) == L
    perms = []
    for l in range(L):
        d = pb.dofs[l]
        assert desc["levels"][l]["n_dof"] == d.n_free, f"level {l}"
        assert len(desc["levels"][l]["cell_ptr"]) - 1 == len(pb.meshes[l].cell_faces)
        pts, knd = g.level_points(l)
        perms.append(_match(pts, knd, d.point[d.free_ids], d.kind[d.free_ids]))
    n = pb.K.shape[0]
    Kn = _assemble(desc, n)
    p0 = perms[0]
    Q = sp.csr_matrix((np.ones(n), (p0, np.arange(n))), shape=(n, n))   # native -> oracle
    assert _rel_rows(Q @ Kn @ Q.T, pb.K) < tol
    # vertices (velocity DOFs)
    vperm = _match(g.vertices, np.zeros(g.n_vert, np.int8), pb.vertices, np.zeros(pb.n_vertices, np.int8))
    V3 = (3 * vperm[:, None] + np.arange(3)[None, :]).ravel()
    nv3 = 3 * g.n_vert
    QV = sp.csr_matrix((np.ones(nv3), (V3, np.arange(nv3))), shape=(nv3, nv3))
    Bn = _assemble_B(desc, n)
    assert _rel_rows(Q @ Bn @ QV.T, pb.B) < tol
    for l in range(L - 1):
        rp, ci, va = desc["levels"][l]["P"]
        nf, nc = desc["levels"][l]["n_dof"], desc["levels"][l + 1]["n_dof"]
        Pn = sp.csr_matrix((va, ci, rp), shape=(nf, nc))
        # structurally equal up to entries that are zero in exact arithmetic
        sig = lambda M: int((np.abs(M.data) > 10 * tol * np.abs(M.data).max()).sum())
        assert sig(Pn) == sig(pb.P[l])
        Qf = sp.csr_matrix((np.ones(nf), (perms[l], np.arange(nf))), shape=(nf, nf))
        Qc = sp.csr_matrix((np.ones(nc), (perms[l + 1], np.arange(nc))), shape=(nc, nc))
        assert _rel_rows(Qf @ Pn @ Qc.T, pb.P[l]) < tol, f"P level {l}"
    # velocity correction: cells matched by centroid, rows per (cell, component, coefficient)
    from oracle import velocity as vel
    ov = vel.operators(pb)
    geom = desc["cell_geom"].reshape(-1, 5)
    ocen = np.array([g_.xc for (_, _, _, g_) in pb.asm.cells])
    dc, cperm = cKDTree(ocen).query(geom[:, :3])
    assert dc.max() < 1e-9 and len(set(cperm.tolist())) == len(cperm)
    nc = len(cperm)
    R12 = (12 * cperm[:, None] + np.arange(12)[None, :]).ravel()
    QC = sp.csr_matrix((np.ones(12 * nc), (R12, np.arange(12 * nc))), shape=(12 * nc, 12 * nc))
    nvv = _velocity_ops(desc, n)
    assert _rel_rows(QC @ nvv["Pi"] @ QV.T, ov["Pi"]) < tol
    assert _rel_rows(QC @ nvv["G"] @ Q.T, ov["G"]) < tol
    assert _rel_rows(QC @ nvv["M"] @ QC.T, ov["M"]) < tol
    assert _rel_rows(QV @ nvv["Av"] @ QC.T, ov["Av"]) < tol
    comp = desc["component"]
    if pb.w.dirichlet_top:
        assert (comp < 0).all()
    else:
        assert desc["n_components"] == len(pb.null.floating)


def test_native_naive_prolongation_matches_oracle():
    """The builder's naive prolongation (Sec. 4 ablation) equals the oracle's, row by row."""
    import synth
    from paper_2607_17725_amd import fvem
    pb = oracle_problem("c3", 8, naive_prolongation=True)
    w = synth.get_config("c3", N=8)
    V, F = w.mesh()
    g = fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top, naive_prolongation=True)
    desc = g.describe()
    L = len(pb.meshes)
    assert len(desc["levels"]) == L
    perms = []
    for l in range(L):
        d = pb.dofs[l]
        assert desc["levels"][l]["n_dof"] == d.n_free, f"level {l}"
        pts, knd = g.level_points(l)
        perms.append(_match(pts, knd, d.point[d.free_ids], d.kind[d.free_ids]))
    for l in range(L - 1):
        rp, ci, va = desc["levels"][l]["P"]
        nf, nc = desc["levels"][l]["n_dof"], desc["levels"][l + 1]["n_dof"]
        Pn = sp.csr_matrix((va, ci, rp), shape=(nf, nc))
        Qf = sp.csr_matrix((np.ones(nf), (perms[l], np.arange(nf))), shape=(nf, nf))
        Qc = sp.csr_matrix((np.ones(nc), (perms[l + 1], np.arange(nc))), shape=(nc, nc))
        assert _rel_rows(Qf @ Pn @ Qc.T, pb.P[l]) < 1e-10, f"P level {l}"
