"""Degrees of freedom and global assembly (Sec. 3.1 eq. for K, Sec. 3.2 for the RHS).

Global DOF numbering of a level (oracle convention): vertices, then edges,
faces and cells (k = 2), each in mesh order.  With a Dirichlet top (z = 1),
the DOFs supported on that face are removed; the free DOFs keep their
relative order.
"""
import numpy as np
import scipy.sparse as sp

from .vem import CellGeometry, element_matrices


class Dofs:
    def __init__(self, mesh, k, dirichlet_top=False):
        self.mesh, self.k = mesh, k
        nv, ne, nf, nc = len(mesh.X), len(mesh.edges), len(mesh.faces), len(mesh.cell_faces)
        self.nv, self.ne, self.nf, self.nc = nv, ne, nf, nc
        self.n = nv if k == 1 else nv + ne + nf + nc
        X = mesh.X
        pts = [X]
        kinds = [np.zeros(nv, dtype=np.int8)]
        if k == 2:
            pts.append(0.5 * (X[mesh.edges[:, 0]] + X[mesh.edges[:, 1]]))
            pts.append(np.array([X[f].mean(axis=0) for f in mesh.faces]))
            pts.append(mesh.cell_centroid)
            kinds += [np.full(ne, 1, np.int8), np.full(nf, 2, np.int8), np.full(nc, 3, np.int8)]
        self.point = np.concatenate(pts)
        self.kind = np.concatenate(kinds)
        top = np.zeros(self.n, dtype=bool)
        if dirichlet_top:
            on = np.abs(X[:, 2] - 1.0) < 1e-12
            top[:nv] = on
            if k == 2:
                top[nv:nv + ne] = on[mesh.edges[:, 0]] & on[mesh.edges[:, 1]]
                top[nv + ne:nv + ne + nf] = [all(on[v] for v in f) for f in mesh.faces]
        self.dirichlet = top
        self.free = np.full(self.n, -1, dtype=np.int64)
        fidx = np.nonzero(~top)[0]
        self.free[fidx] = np.arange(len(fidx))
        self.n_free = len(fidx)
        self.free_ids = fidx

    def deactivate(self, dof_ids):
        """Remove DOFs from the free set (coarse DOFs the prolongation never uses)."""
        self.dirichlet = self.dirichlet.copy()
        self.inactive = np.zeros(self.n, dtype=bool) if not hasattr(self, "inactive") else self.inactive
        self.inactive[dof_ids] = True
        keep = ~(self.dirichlet | self.inactive)
        self.free = np.full(self.n, -1, dtype=np.int64)
        fidx = np.nonzero(keep)[0]
        self.free[fidx] = np.arange(len(fidx))
        self.n_free = len(fidx)
        self.free_ids = fidx

    def cell_dofs(self, c):
        m = self.mesh
        out = list(m.cell_verts[c])
        if self.k == 2:
            out += [self.nv + e for e in m.cell_edges[c]]
            out += [self.nv + self.ne + f for f in m.cell_face_ids[c]]
            out.append(self.nv + self.ne + self.nf + c)
        return np.array(out, dtype=np.int64)


def _shape_key(g, k, h):
    """Exact key for cells whose vertices sit on the background lattice, else None.

    Such cells (uncut cubes and their aggregates) share element matrices with
    every translate; all other cells are computed one by one.
    """
    X = g.X
    base = X[g.verts].min(axis=0)
    key = [k]
    for cyc in g.faces:
        rel = (X[cyc] - base) / h
        r = np.rint(rel)
        if np.abs(rel - r).max() > 1e-12:
            return None
        key.append(tuple(r.astype(np.int64).ravel()))
    return tuple(key)


class Assembly:
    """Element data and assembled operators of the finest level."""

    def __init__(self, mesh, dofs, with_velocity=True):
        k = dofs.k
        cache = {}
        self.cells = []
        rows, cols, vals = [], [], []
        brow, bcol, bval = [], [], []
        for c in range(len(mesh.cell_faces)):
            g = CellGeometry(mesh, c)
            key = _shape_key(g, k, mesh.h)
            em = cache.get(key) if key is not None else None
            if em is None:
                em = element_matrices(g, k, with_velocity)
                if key is not None:
                    cache[key] = em
            gd = dofs.cell_dofs(c)
            self.cells.append((gd, np.array(g.verts), em, g))
            fd = dofs.free[gd]
            keep = fd >= 0
            K = em["K"][np.ix_(keep, keep)]
            r = np.repeat(fd[keep], keep.sum())
            cc = np.tile(fd[keep], keep.sum())
            rows.append(r)
            cols.append(cc)
            vals.append(K.ravel())
            if with_velocity:
                vc = (3 * np.array(g.verts)[:, None] + np.arange(3)[None, :]).ravel()
                Bm = em["B"][keep]
                brow.append(np.repeat(fd[keep], len(vc)))
                bcol.append(np.tile(vc, keep.sum()))
                bval.append(Bm.ravel())
        n = dofs.n_free
        self.K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        self.K.sum_duplicates()
        self.K.sort_indices()
        if with_velocity:
            self.B = sp.csr_matrix((np.concatenate(bval), (np.concatenate(brow), np.concatenate(bcol))),
                                   shape=(n, 3 * dofs.nv))
            self.B.sum_duplicates()
            self.B.sort_indices()
        self.n_shapes = len(cache)

    def project_velocity(self, dofs, u, p_free):
        """Per cell 3x4 coefficients of Pi_1 u - grad(Pi_k p) (Sec. 3.3)."""
        p = np.zeros(dofs.n)
        p[dofs.free_ids] = p_free
        out = np.zeros((len(self.cells), 3, 4))
        U = u.reshape(-1, 3)
        for c, (gd, verts, em, g) in enumerate(self.cells):
            for d in range(3):
                out[c, d] = em["Pi1s"] @ U[verts, d] - em["CPis"][d] @ p[gd]
        return out

    def loss(self, s, t):
        """sum_E int_E |s_E - t_E|^2 with the cell mass matrix of linear monomials."""
        tot = 0.0
        for c, (gd, verts, em, g) in enumerate(self.cells):
            d = s[c] - t[c]
            tot += float(np.einsum("ia,ab,ib->", d, em["M1"], d))
        return tot

    def pi1(self, u):
        out = np.zeros((len(self.cells), 3, 4))
        U = u.reshape(-1, 3)
        for c, (gd, verts, em, g) in enumerate(self.cells):
            for d in range(3):
                out[c, d] = em["Pi1s"] @ U[verts, d]
        return out


def components(A):
    """Connected components of the matrix graph (labels per row)."""
    from scipy.sparse.csgraph import connected_components
    return connected_components(A, directed=False)[1]
