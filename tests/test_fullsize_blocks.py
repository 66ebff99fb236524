"""Element blocks of the native builder at 128^3 against the oracle, cell by cell.

For the benchmark's plates (c3) and the 1e-5-thin sheet (c4) at their full
128^3 size, 200 seeded cut cells and the 50 smallest cells (the sheet's
slivers) are taken from the native grid.  The oracle rebuilds each cell's
VEM stiffness K^E and divergence block B^E from the cell's outward face
polygons alone (its own projector, quadrature and monomial frames), and the
blocks must agree entry by entry after matching local DOFs by (kind, support
point) and velocity vertices by position: 1e-10 of the row's largest entry,
1e-6 on the sheet (the bounds of the 8^3 builder parity test).

The test needs no GPU: it is kept with the GPU suite because the two full
size grid builds take minutes of host time, beyond the CPU suite's budget.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle.vem import StandaloneCell, element_matrices

pytestmark = pytest.mark.gpu


def _rel_rows(A, B):
    scale = np.maximum(np.abs(B).max(axis=1), 1e-300)
    return float((np.abs(A - B).max(axis=1) / scale).max())


@pytest.mark.parametrize("name,tol", [("c3", 1e-10), ("c4", 1e-6)])
def test_sampled_cut_cell_blocks_at_full_size(name, tol):
    import synth
    from paper_2607_17725_amd import fvem
    w = synth.get_config(name)
    V, F = w.mesh()
    print(f"[fullsize blocks] building {name} at {w.N}^3 on the host", flush=True)
    g = fvem.Grid(V, F, w.N, w.k, w.levels, w.dirichlet_top)
    d = g.describe()
    lv = d["levels"][0]
    cp, cd = lv["cell_ptr"], lv["cell_dof"]
    nc = len(cp) - 1
    geom = d["cell_geom"].reshape(nc, 5)
    ke_off, be_off = d["ke_off"], d["be_off"]
    # cut (and otherwise irregular) cells own their blocks; uncut cubes share one
    off, count = np.unique(ke_off, return_counts=True)
    own = np.isin(ke_off, off[count == 1])
    cut = np.nonzero(own)[0]
    rng = np.random.default_rng(11)
    sample = np.union1d(rng.choice(cut, size=min(200, len(cut)), replace=False),
                        cut[np.argsort(geom[cut, 4])[:50]])
    print(f"[fullsize blocks] {name}: {nc} cells, {len(cut)} cut, {len(sample)} sampled, "
          f"smallest volume {geom[cut, 4].min():.2e}", flush=True)
    worst_k = worst_b = 0.0
    for c in sample:
        faces = g.cell_faces(c)
        cell = StandaloneCell([g.vertices[f] for f in faces])
        em = element_matrices(cell, w.k)
        X = cell.X
        nv, ne, nf = len(cell.verts), len(cell.edges), len(cell.faces)
        pts = [X[cell.verts], np.array([0.5 * (X[a] + X[b]) for a, b in cell.edge_pairs]),
               np.array([X[f].mean(axis=0) for f in cell.faces]), cell.xc[None, :]]
        kinds = np.repeat([0, 1, 2, 3], [nv, ne, nf, 1])
        if w.k == 1:
            pts, kinds = pts[:1], kinds[:nv]
        pts = np.concatenate(pts)
        dofs = cd[cp[c]:cp[c + 1]]
        assert np.all(dofs >= 0) and len(dofs) == len(pts)
        perm = np.full(len(dofs), -1)
        for kind in range(4):
            a = np.nonzero(g.dof_kind[dofs] == kind)[0]
            b = np.nonzero(kinds == kind)[0]
            assert len(a) == len(b)
            if len(a):
                dist, j = cKDTree(pts[b]).query(g.dof_points[dofs[a]])
                assert dist.max() < 1e-9
                perm[a] = b[j]
        assert len(set(perm.tolist())) == len(perm)
        m = len(dofs)
        Kb = d["ke_val"][ke_off[c]:ke_off[c] + m * m].reshape(m, m)
        worst_k = max(worst_k, _rel_rows(Kb, em["K"][np.ix_(perm, perm)]))
        verts = d["cell_vert"][d["cell_vptr"][c]:d["cell_vptr"][c + 1]]
        dist, vj = cKDTree(X[cell.verts]).query(g.vertices[verts])
        assert dist.max() < 1e-12
        cols = (3 * vj[:, None] + np.arange(3)[None, :]).ravel()
        Bb = d["be_val"][be_off[c]:be_off[c] + m * 3 * len(verts)].reshape(m, 3 * len(verts))
        worst_b = max(worst_b, _rel_rows(Bb, em["B"][np.ix_(perm, cols)]))
    print(f"[fullsize blocks] {name}: worst row error K {worst_k:.2e}, B {worst_b:.2e}", flush=True)
    assert worst_k <= tol and worst_b <= tol
