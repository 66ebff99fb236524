"""Diffusion-free VEM prolongation (Sec. 4, "Diffusion-Free VEM Prolongation Operator").

A fine DOF that coincides with a coarse DOF copies it.  Every other fine DOF
is evaluated from the coarse function's projection on the lowest-dimensional
coarse entity whose closure holds the DOF's support:
* a coarse edge: the 1-D space is P_k(e) itself, so the projection is the
  Lagrange interpolant through the edge's DOFs;
* a coarse face: the 2-D projection Pi_f of the face's own DOFs;
* a coarse cell: the 3-D projection Pi of the cell's DOFs.
Point DOFs (vertices, edge midpoints) take the projection's value at the
point; face-mean and cell-mean DOFs take its mean over the fine face / cell.
Because every fine DOF of a fine cell inside coarse cell E depends on DOFs of
E only, the Galerkin product couples only DOFs of one coarse cell.

Reading for the set notation the paper leaves garbled: the new fine DOFs are
split by the dimension of their host entity, which makes the edge, face and
volume sets pairwise disjoint.  Coarse DOFs on a Dirichlet face are dropped
(their value is zero).  Coarse DOFs that no fine DOF depends on give zero
columns; the caller drops them, so the coarse operators stay non-singular.
That is this build's reading, not the paper's: Sec. 5.2 argues nestedness
avoids rank-deficient transfers, but coarse cells here keep their solid part
(the coarse-inclusion reading), which leaves such DOFs.
"""
import numpy as np
import scipy.sparse as sp

from .quadrature import polygon_rule, polyhedron_rule
from .vem import CellGeometry, cell_projector, face_projector

TOL = 1e-9
# a point lies on a coarse vertex or edge within the vertex weld distance of
# the mesh (points that do are there up to rounding; 1e-9 took a fine edge
# midpoint 9e-9 from a coarse vertex for a point of a neighbouring edge)
POINT_TOL = 1e-10
WEIGHT_TOL = 1e-13


def _point_in_face(p, P, n, tol=TOL):
    d = float(n @ P[0])
    if abs(float(n @ p) - d) > tol:
        return False
    m = len(P)
    Q = np.roll(P, -1, axis=0)
    E = Q - P
    on = np.stack([E[:, 1] * n[2] - E[:, 2] * n[1], E[:, 2] * n[0] - E[:, 0] * n[2],
                   E[:, 0] * n[1] - E[:, 1] * n[0]], -1)
    s = np.einsum("ij,ij->i", on, p - P)
    return bool(np.all(s <= tol * np.sqrt((on ** 2).sum(1))))


class CoarseLevel:
    """Lazily computed projections of a coarse level."""

    def __init__(self, mesh, dofs):
        self.mesh, self.dofs = mesh, dofs
        self.k = dofs.k
        self._cell = {}
        self._face = {}

    def cell(self, c):
        if c not in self._cell:
            g = CellGeometry(self.mesh, c)
            Pis, _, _ = cell_projector(g, self.k)
            self._cell[c] = (g, Pis, self.dofs.cell_dofs(c))
        return self._cell[c]

    def face(self, f):
        """(Pi_f*, frame, global coarse DOFs of the face in face-local order)."""
        if f not in self._face:
            m = self.mesh
            cyc = m.faces[f]
            P = m.X[cyc]
            Pif, fr = face_projector(P, m.face_normal[f], self.k)
            gd = list(cyc)
            if self.k == 2:
                nv, ne = self.dofs.nv, self.dofs.ne
                for i in range(len(cyc)):
                    a, b = cyc[i], cyc[(i + 1) % len(cyc)]
                    gd.append(nv + m.edge_index[(a, b) if a < b else (b, a)])
                gd.append(nv + ne + f)
            self._face[f] = (Pif, fr, np.array(gd))
        return self._face[f]


class _CellContainment:
    """Coarse cells whose closure holds a point or a fine face (naive prolongation)."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.planes = []
        for c in range(len(mesh.cell_faces)):
            pl = []
            for f, o in mesh.cell_faces[c]:
                n = mesh.face_normal[f] * o
                pl.append((n, float(n @ mesh.X[mesh.faces[f][0]])))
            self.planes.append(pl)
        self.vert_cells = {}
        for c in range(len(mesh.cell_faces)):
            for v in mesh.cell_verts[c]:
                self.vert_cells.setdefault(int(v), []).append(c)

    def cells_holding(self, pts, E, tol=TOL):
        """Cells (E first, then increasing id) whose closure holds every point of pts."""
        cand = sorted({c for v in self.mesh.cell_verts[E] for c in self.vert_cells[int(v)]} - {E})
        out = [E]
        for c in cand:
            if all(float(n @ p) <= d + tol for n, d in self.planes[c] for p in pts):
                out.append(c)
        return out


def build_prolongation(fine_mesh, fine_dofs, coarse_mesh, coarse_dofs, parent, return_raw=False, naive=False):
    """P [fine free x coarse free] as scipy CSR, plus the host kind per fine DOF.

    With ``return_raw`` also the prolongation before rounding-level weights
    are dropped (every coarse column kept).  With ``naive`` the naive VEM
    prolongation of Sec. 4 instead: DOFs shared with the coarse level (same
    vertex, edge, face or cell) copy it, and every other fine DOF takes the
    DOF functional of the coarse cell projection Pi_k; a DOF on the boundary
    of several coarse cells takes the mean of their projections (the
    reading for a face or edge shared by coarse cells, which the paper
    leaves open).  Rows then reach DOFs of neighbouring coarse cells, the
    connectivity diffusion the diffusion-free operator avoids.
    """
    k = fine_dofs.k
    CL = coarse_level = CoarseLevel(coarse_mesh, coarse_dofs)
    X, Xc = fine_mesh.X, coarse_mesh.X
    nvf, nef, nff = fine_dofs.nv, fine_dofs.ne, fine_dofs.nf
    rows = {}
    host_kind = np.full(fine_dofs.n, -1, dtype=np.int8)
    cont = _CellContainment(coarse_mesh) if naive else None

    def mean_rows(parts):
        out = {}
        for row in parts:
            for j, w in row.items():
                out[j] = out.get(j, 0.0) + w / len(parts)
        return out

    def naive_point_row(p, E):
        g, Pis, cd = CL.cell(E)
        for v in g.verts:
            if np.linalg.norm(Xc[v] - p) < POINT_TOL:
                return {int(v): 1.0}, 0
        if k == 2:
            for e in g.edges:
                a, b = coarse_mesh.edges[e]
                if np.linalg.norm(0.5 * (Xc[a] + Xc[b]) - p) < POINT_TOL:
                    return {int(coarse_dofs.nv + e): 1.0}, 1
        parts = []
        for c in cont.cells_holding([p], E):
            gc, Pc, cdc = CL.cell(c)
            parts.append(dict(zip(cdc.tolist(), (gc.basis.mono(p, k)[0] @ Pc).tolist())))
        return mean_rows(parts), 3

    def naive_face_mean_row(fpts, E):
        g, Pis, cd = CL.cell(E)
        qp, qw = polygon_rule(fpts)
        area_f = qw.sum()
        fc = qw @ qp / area_f
        for f in g.face_ids:
            P = Xc[coarse_mesh.faces[f]]
            n = coarse_mesh.face_normal[f]
            qpc, qwc = polygon_rule(P)
            if np.abs((fpts - P[0]) @ n).max() <= TOL and abs(qwc.sum() - area_f) < 1e-12 * area_f and \
                    np.linalg.norm(qwc @ qpc / qwc.sum() - fc) < TOL:
                return {int(coarse_dofs.nv + coarse_dofs.ne + f): 1.0}, 4
        parts = []
        for c in cont.cells_holding(fpts, E):
            gc, Pc, cdc = CL.cell(c)
            parts.append(dict(zip(cdc.tolist(), ((qw @ gc.basis.mono(qp, k) / area_f) @ Pc).tolist())))
        return mean_rows(parts), 3

    def point_row(p, E):
        g, Pis, cd = CL.cell(E)
        # coarse vertex
        for v in g.verts:
            if np.linalg.norm(Xc[v] - p) < POINT_TOL:
                return {int(v): 1.0}, 0
        # coarse edge
        for e in g.edges:
            a, b = coarse_mesh.edges[e]
            pa, pb = Xc[a], Xc[b]
            ab = pb - pa
            tau = float((p - pa) @ ab / (ab @ ab))
            if 0.0 < tau < 1.0 and np.linalg.norm(p - pa - tau * ab) < POINT_TOL:
                if k == 1:
                    return {int(a): 1.0 - tau, int(b): tau}, 1
                mid = coarse_dofs.nv + e
                return {int(a): 2 * (tau - 0.5) * (tau - 1.0), int(mid): -4.0 * tau * (tau - 1.0),
                        int(b): 2.0 * tau * (tau - 0.5)}, 1
        # coarse face
        for f in g.face_ids:
            P = Xc[coarse_mesh.faces[f]]
            if _point_in_face(p, P, coarse_mesh.face_normal[f]):
                Pif, fr, fd = CL.face(f)
                w = fr.mono(p, k)[0] @ Pif
                return dict(zip(fd.tolist(), w.tolist())), 2
        w = g.basis.mono(p, k)[0] @ Pis
        return dict(zip(cd.tolist(), w.tolist())), 3

    def face_mean_row(fpts, E):
        g, Pis, cd = CL.cell(E)
        qp, qw = polygon_rule(fpts)
        area_f = qw.sum()
        fc = qw @ qp / area_f
        # the fine face lies in the coarse face's plane when all of its
        # vertices do (a distance test: the computed normal of a sliver face
        # can be off by far more than its vertices are)
        coplanar = []
        for f in g.face_ids:
            P = Xc[coarse_mesh.faces[f]]
            n = coarse_mesh.face_normal[f]
            if np.abs((fpts - P[0]) @ n).max() <= TOL:
                coplanar.append((f, P, n))
        # a coarse face equal to the fine face is its host before any face the
        # fine face's centroid is merely near (a tiny fine face beside a
        # coarse edge passes the containment slack of the neighbouring face)
        for f, P, n in coplanar:
            qpc, qwc = polygon_rule(P)
            if abs(qwc.sum() - area_f) < 1e-12 * area_f and \
                    np.linalg.norm(qwc @ qpc / qwc.sum() - fc) < TOL:
                return {int(coarse_dofs.nv + coarse_dofs.ne + f): 1.0}, 4
        for f, P, n in coplanar:
            if not _point_in_face(fc, P, n):
                continue
            Pif, fr, fd = CL.face(f)
            w = (qw @ fr.mono(qp, k) / area_f) @ Pif
            return dict(zip(fd.tolist(), w.tolist())), 2
        w = (qw @ g.basis.mono(qp, k) / area_f) @ Pis
        return dict(zip(cd.tolist(), w.tolist())), 3

    def cell_mean_row(c_f, E):
        g, Pis, cd = CL.cell(E)
        vol_f = fine_mesh.cell_volume[c_f]
        if abs(vol_f - coarse_mesh.cell_volume[E]) < 1e-12 * vol_f and \
                np.linalg.norm(fine_mesh.cell_centroid[c_f] - coarse_mesh.cell_centroid[E]) < TOL:
            return {int(cd[-1]): 1.0}, 4
        gf = CellGeometry(fine_mesh, c_f)
        qp, qw = polyhedron_rule([X[c] for c in gf.faces], centre=X[gf.verts].mean(axis=0))
        w = (qw @ g.basis.mono(qp, k) / qw.sum()) @ Pis
        return dict(zip(cd.tolist(), w.tolist())), 3

    if naive:
        point_row, face_mean_row = naive_point_row, naive_face_mean_row
    for c in range(len(fine_mesh.cell_faces)):
        E = int(parent[c])
        fd = fine_dofs.cell_dofs(c)
        for v in fine_mesh.cell_verts[c]:
            if v not in rows:
                rows[v], host_kind[v] = point_row(X[v], E)
        if k == 2:
            for e in fine_mesh.cell_edges[c]:
                i = nvf + e
                if i not in rows:
                    a, b = fine_mesh.edges[e]
                    rows[i], host_kind[i] = point_row(0.5 * (X[a] + X[b]), E)
            for f in fine_mesh.cell_face_ids[c]:
                i = nvf + nef + f
                if i not in rows:
                    rows[i], host_kind[i] = face_mean_row(X[fine_mesh.faces[f]], E)
            i = nvf + nef + nff + c
            rows[i], host_kind[i] = cell_mean_row(c, E)
    r, cidx, val, keep = [], [], [], []
    for i, row in rows.items():
        fi = fine_dofs.free[i]
        if fi < 0:
            continue
        # weights at rounding level of the row's largest weight are exact
        # zeros of the prolongation (a projection evaluated where a basis
        # function's contribution cancels, e.g. DOFs of coplanar sub-faces
        # of a split coarse face); keeping their rounding residue would leave
        # coarse DOFs with numerically empty columns and near-zero coarse
        # diagonals.  The pins show the dropped weights are exact zeros and
        # sit at least five orders of magnitude below every kept weight.
        wmax = max((abs(w) for w in row.values()), default=0.0)
        for j, w in row.items():
            cj = coarse_dofs.free[j]
            if cj < 0:
                continue
            r.append(fi)
            cidx.append(cj)
            val.append(w)
            keep.append(abs(w) > WEIGHT_TOL * wmax)
    r, cidx, val, keep = map(np.asarray, (r, cidx, val, keep))
    shape = (fine_dofs.n_free, coarse_dofs.n_free)
    P_raw = sp.csr_matrix((val, (r, cidx)), shape=shape)
    P_raw.sum_duplicates()
    P_raw.sort_indices()
    P = sp.csr_matrix((val[keep], (r[keep], cidx[keep])), shape=shape)
    P.sum_duplicates()
    P.sort_indices()
    if return_raw:
        return P, host_kind, P_raw
    return P, host_kind
