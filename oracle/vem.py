"""Conforming virtual elements of order k = 1, 2 on convex polyhedra (Sec. 3.1, App. A).

Local degrees of freedom of a cell E, in this order: vertex values, values at
edge midpoints (k = 2; the single interior Gauss-Lobatto point), face means
(k = 2), the cell mean (k = 2).

Scaled monomials m_a((x - x_E)/h_E) with x_E the volume centroid and h_E the
largest vertex distance, ordered 1, x, y, z, x^2, xy, xz, y^2, yz, z^2.

The projector Pi (the H1 projection onto polynomials) solves the orthogonality
conditions plus the P0 constraint (vertex mean for k = 1, cell mean for
k = 2).  Its right-hand side integrates by parts:
    int_E grad(phi).grad(m) = -int_E phi lap(m) + sum_f int_f phi grad(m).n_f,
where the cell term uses the cell-mean DOF (lap m is constant for k <= 2) and
the face term uses the face space's own projection,
    int_f phi q = int_f Pi_f(phi) q  for polynomial q of degree <= k-1,
(the standard enhanced face space; the paper obtains the face and edge
projections "by dimensional reduction").  On an edge a function of the space is
the degree-k polynomial through its DOFs, so the edge integrals of Pi_f's
right-hand side are exact with the trapezoid (k = 1) or Simpson (k = 2) rule.

Element stiffness: consistency term plus the DOF-based ("dofi-dofi")
stabilisation, the latter scaled by h_E so both terms scale alike in 3-D
(reading; the paper cites the 2-D theory, where the scale is 1).

Divergence right-hand side (Sec. 3.2): the velocity is the first-order field
with vertex values; b_r = sum_E int_E Pi_1(u) . grad(Pi_k phi_r) (reading of
the paper's projected right-hand side; it matches the gradient used by the
grid-to-particle update).
"""
import numpy as np

from .geometry import cross3, norm3, polygon_area_vec
from .quadrature import polygon_rule, polyhedron_rule

EXP3 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
        (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]
EXP2 = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def n_poly3(k):
    return 4 if k == 1 else 10


def n_poly2(k):
    return 3 if k == 1 else 6


def mono3(X, xc, hc, k):
    """[Q, N_k] values of the scaled monomials at points X [Q,3]."""
    Y = (np.atleast_2d(X) - xc) / hc
    return np.stack([Y[:, 0] ** a * Y[:, 1] ** b * Y[:, 2] ** c for a, b, c in EXP3[:n_poly3(k)]], -1)


def grad_mono3(X, xc, hc, k):
    """[Q, N_k, 3] gradients of the scaled monomials."""
    Y = (np.atleast_2d(X) - xc) / hc
    out = np.zeros((len(Y), n_poly3(k), 3))
    for i, (a, b, c) in enumerate(EXP3[:n_poly3(k)]):
        if a:
            out[:, i, 0] = a * Y[:, 0] ** (a - 1) * Y[:, 1] ** b * Y[:, 2] ** c / hc
        if b:
            out[:, i, 1] = b * Y[:, 0] ** a * Y[:, 1] ** (b - 1) * Y[:, 2] ** c / hc
        if c:
            out[:, i, 2] = c * Y[:, 0] ** a * Y[:, 1] ** b * Y[:, 2] ** (c - 1) / hc
    return out


def lap_mono3(hc, k):
    out = np.zeros(n_poly3(k))
    for i, (a, b, c) in enumerate(EXP3[:n_poly3(k)]):
        out[i] = (a * (a - 1) + b * (b - 1) + c * (c - 1)) / hc ** 2
    return out


def deriv_to_linear(hc, k):
    """C[c] (4 x N_k): d/dx_c of each monomial in the linear monomial basis."""
    C = np.zeros((3, 4, n_poly3(k)))
    lin = {e: i for i, e in enumerate(EXP3[:4])}
    for j, e in enumerate(EXP3[:n_poly3(k)]):
        for c in range(3):
            if e[c] == 0:
                continue
            r = list(e)
            r[c] -= 1
            C[c, lin[tuple(r)], j] = e[c] / hc
    return C


ANISO_RATIO = 4.0


class Basis3:
    """Monomials of y = R^T (x - x_c) / s up to degree k.

    The paper's basis is R = I, s = (h_E, h_E, h_E).  Thin cells (principal
    extents differing by more than ANISO_RATIO) use their principal axes and
    per-axis half-extents instead: the projection is the same polynomial in
    any basis of P_k, but the isotropic basis makes the local systems of a
    1e-5-thin cell singular to working precision.
    """

    def __init__(self, X, xc, hc):
        self.xc = xc
        D = X - xc
        _, sv, Vt = np.linalg.svd(D, full_matrices=False)
        if sv[0] > ANISO_RATIO * sv[-1]:
            self.R = Vt.T
            self.s = np.abs(D @ self.R).max(axis=0)
        else:
            self.R = np.eye(3)
            self.s = np.full(3, hc)
        self.hc = hc

    def local(self, X):
        return ((np.atleast_2d(X) - self.xc) @ self.R) / self.s

    def mono(self, X, k):
        Y = self.local(X)
        return np.stack([Y[:, 0] ** a * Y[:, 1] ** b * Y[:, 2] ** c for a, b, c in EXP3[:n_poly3(k)]], -1)

    def grad(self, X, k):
        Y = self.local(X)
        dy = np.zeros((len(Y), n_poly3(k), 3))
        for i, (a, b, c) in enumerate(EXP3[:n_poly3(k)]):
            if a:
                dy[:, i, 0] = a * Y[:, 0] ** (a - 1) * Y[:, 1] ** b * Y[:, 2] ** c
            if b:
                dy[:, i, 1] = b * Y[:, 0] ** a * Y[:, 1] ** (b - 1) * Y[:, 2] ** c
            if c:
                dy[:, i, 2] = c * Y[:, 0] ** a * Y[:, 1] ** b * Y[:, 2] ** (c - 1)
        return np.einsum("qnc,c,ic->qni", dy, 1.0 / self.s, self.R)

    def lap(self, k):
        s2 = self.s ** 2
        return np.array([a * (a - 1) / s2[0] + b * (b - 1) / s2[1] + c * (c - 1) / s2[2]
                         for a, b, c in EXP3[:n_poly3(k)]])

    def deriv_to_linear(self, k):
        """C[c] (4 x N_k): d/dx_c of each basis polynomial in this basis's linear part."""
        Cy = np.zeros((3, 4, n_poly3(k)))          # d/dy_d
        lin = {e: i for i, e in enumerate(EXP3[:4])}
        for j, e in enumerate(EXP3[:n_poly3(k)]):
            for d in range(3):
                if e[d] == 0:
                    continue
                r = list(e)
                r[d] -= 1
                Cy[d, lin[tuple(r)], j] = e[d]
        # d/dx_c = sum_d R[c, d] / s_d d/dy_d
        return np.einsum("cd,d,dij->cij", self.R, 1.0 / self.s, Cy)

    def linear_to_paper(self):
        """T (4x4): coefficients on [1, y] -> coefficients on the paper's [1, (x - x_c)/h_E]."""
        T = np.zeros((4, 4))
        T[0, 0] = 1.0
        T[1:, 1:] = self.R * (self.hc / self.s)[None, :]
        return T


class FaceFrame:
    def __init__(self, P, n):
        self.P = P
        self.n = n
        o = P[0]
        U, W = P[1:-1] - o, P[2:] - o
        t = 0.5 * np.stack([U[:, 1] * W[:, 2] - U[:, 2] * W[:, 1], U[:, 2] * W[:, 0] - U[:, 0] * W[:, 2],
                            U[:, 0] * W[:, 1] - U[:, 1] * W[:, 0]], -1) @ n
        self.area = float(t.sum())
        self.xc = o + (t[:, None] * (U + W)).sum(0) / (3.0 * self.area)
        d = P[:, None, :] - P[None, :, :]
        self.hc = float(np.sqrt((d ** 2).sum(-1).max()))
        t1 = P[1] - P[0]
        self.t1 = t1 / norm3(t1)
        self.t2 = cross3(n, self.t1)
        Q = np.stack([(P - self.xc) @ self.t1, (P - self.xc) @ self.t2], -1)
        _, sv, Vt = np.linalg.svd(Q, full_matrices=False)
        if sv[0] > ANISO_RATIO * sv[-1]:
            a1 = Vt[0, 0] * self.t1 + Vt[0, 1] * self.t2
            a1 /= norm3(a1)
            self.t1 = a1
            self.t2 = cross3(n, a1)
            Q = np.stack([(P - self.xc) @ self.t1, (P - self.xc) @ self.t2], -1)
            self.s = np.abs(Q).max(axis=0)
        else:
            self.s = np.array([self.hc, self.hc])

    def local(self, X):
        D = np.atleast_2d(X) - self.xc
        return np.stack([D @ self.t1, D @ self.t2], -1) / self.s

    def mono(self, X, k):
        Y = self.local(X)
        return np.stack([Y[:, 0] ** a * Y[:, 1] ** b for a, b in EXP2[:n_poly2(k)]], -1)

    def grad_mono(self, X, k):
        """[Q, N, 3] 3-D (in-plane) gradients of the face monomials."""
        Y = self.local(X)
        out = np.zeros((len(Y), n_poly2(k), 3))
        for i, (a, b) in enumerate(EXP2[:n_poly2(k)]):
            gs = a * Y[:, 0] ** max(a - 1, 0) * Y[:, 1] ** b / self.s[0] if a else 0 * Y[:, 0]
            gt = b * Y[:, 0] ** a * Y[:, 1] ** max(b - 1, 0) / self.s[1] if b else 0 * Y[:, 0]
            out[:, i, :] = gs[:, None] * self.t1 + gt[:, None] * self.t2
        return out

    def lap_mono(self, k):
        return np.array([a * (a - 1) / self.s[0] ** 2 + b * (b - 1) / self.s[1] ** 2
                         for a, b in EXP2[:n_poly2(k)]])


def face_projector(P, n, k):
    """Pi_f* [N_f x n_f]: monomial coefficients of the face projection.

    Face DOFs: vertices (m), edge midpoints (m, k = 2), face mean (k = 2).
    """
    fr = FaceFrame(P, n)
    m = len(P)
    nd = m if k == 1 else 2 * m + 1
    Nf = n_poly2(k)
    qp, qw = polygon_rule(P)
    D = np.zeros((nd, Nf))
    D[:m] = fr.mono(P, k)
    if k == 2:
        mids = 0.5 * (P + np.roll(P, -1, axis=0))
        D[m:2 * m] = fr.mono(mids, k)
        D[2 * m] = qw @ fr.mono(qp, k) / fr.area
    B = np.zeros((Nf, nd))
    if k == 1:
        B[0, :m] = 1.0 / m
    else:
        B[0, 2 * m] = 1.0
        B[:, 2 * m] += -fr.lap_mono(k) * fr.area
    for i in range(m):
        a, b = P[i], P[(i + 1) % m]
        L = norm3(b - a)
        ne = cross3(b - a, n) / L
        ga = fr.grad_mono(a, k)[0] @ ne
        gb = fr.grad_mono(b, k)[0] @ ne
        if k == 1:
            B[1:, i] += 0.5 * L * ga[1:]
            B[1:, (i + 1) % m] += 0.5 * L * gb[1:]
        else:
            gm = fr.grad_mono(0.5 * (a + b), k)[0] @ ne
            B[1:, i] += L / 6.0 * ga[1:]
            B[1:, m + i] += 4.0 * L / 6.0 * gm[1:]
            B[1:, (i + 1) % m] += L / 6.0 * gb[1:]
    G = B @ D
    return np.linalg.solve(G, B), fr


class CellGeometry:
    """Geometry of one cell: vertex/edge/face lists (global ids) and coordinates."""

    def __init__(self, mesh, c):
        self.verts = list(mesh.cell_verts[c])
        self.edges = list(mesh.cell_edges[c])
        self.face_ids = list(mesh.cell_face_ids[c])
        self.faces = [mesh.faces[f] if o > 0 else mesh.faces[f][::-1] for f, o in mesh.cell_faces[c]]
        self.X = mesh.X
        self.volume = mesh.cell_volume[c]
        self.xc = mesh.cell_centroid[c]
        V = mesh.X[self.verts]
        d = V[:, None, :] - V[None, :, :]
        self.hc = float(np.sqrt((d ** 2).sum(-1).max()))
        self.basis = Basis3(V, self.xc, self.hc)
        self.vloc = {v: i for i, v in enumerate(self.verts)}
        self.eloc = {e: i for i, e in enumerate(self.edges)}
        self.edge_pairs = [tuple(mesh.edges[e]) for e in self.edges]
        self.edge_index = mesh.edge_index

    def n_local(self, k):
        if k == 1:
            return len(self.verts)
        return len(self.verts) + len(self.edges) + len(self.faces) + 1


def cell_projector(g, k):
    """Return (Pi* [N_k x n_E], D [n_E x N_k], G [N_k x N_k]) for cell geometry g."""
    X = g.X
    nv, ne, nf = len(g.verts), len(g.edges), len(g.faces)
    nE = g.n_local(k)
    Nk = n_poly3(k)
    faces_pts = [X[cyc] for cyc in g.faces]
    qp, qw = polyhedron_rule(faces_pts, centre=X[g.verts].mean(axis=0))
    bs = g.basis
    D = np.zeros((nE, Nk))
    D[:nv] = bs.mono(X[g.verts], k)
    B = np.zeros((Nk, nE))
    if k == 1:
        B[0, :nv] = 1.0 / nv
    else:
        mids = np.array([0.5 * (X[a] + X[b]) for a, b in g.edge_pairs])
        D[nv:nv + ne] = bs.mono(mids, k)
        D[nE - 1] = qw @ bs.mono(qp, k) / g.volume
        B[0, nE - 1] = 1.0
        B[:, nE - 1] += -bs.lap(k) * g.volume
    for fi, cyc in enumerate(g.faces):
        P = X[cyc]
        nvec = polygon_area_vec(P)
        nvec /= norm3(nvec)
        Pif, fr = face_projector(P, nvec, k)
        fp, fw = polygon_rule(P)
        gn = bs.grad(fp, k) @ nvec                            # [Q, N_k]
        I = (fr.mono(fp, k) * fw[:, None]).T @ gn             # [N_f, N_k]
        contrib = (Pif.T @ I).T                               # [N_k, n_fdofs]
        m = len(cyc)
        loc = [g.vloc[v] for v in cyc]
        if k == 2:
            for i in range(m):
                a, b = cyc[i], cyc[(i + 1) % m]
                loc.append(nv + g.eloc[g.edge_index[(a, b) if a < b else (b, a)]])
            loc.append(nv + ne + fi)
            D[nv + ne + fi] = (fw @ bs.mono(fp, k)) / fw.sum()
        for j, L in enumerate(loc):
            B[1:, L] += contrib[1:, j]
    G = B @ D
    Pis = np.linalg.solve(G, B)
    return Pis, D, G


def element_matrices(g, k, with_velocity=True):
    """K^E, and (if asked) the divergence block B^E [n_E, n_v*3], Pi_k*, Pi_1*, mass."""
    Pis, D, G = cell_projector(g, k)
    nE = D.shape[0]
    Gt = G.copy()
    Gt[0, :] = 0.0
    Pi = D @ Pis
    IP = np.eye(nE) - Pi
    K = Pis.T @ Gt @ Pis + g.hc * IP.T @ IP
    out = {"K": K, "Pis": Pis}
    if with_velocity:
        Pi1 = Pis if k == 1 else cell_projector(g, 1)[0]
        X = g.X
        qp, qw = polyhedron_rule([X[c] for c in g.faces], centre=X[g.verts].mean(axis=0))
        bs = g.basis
        m1 = bs.mono(qp, 1)                           # [Q,4]
        gk = bs.grad(qp, k)                           # [Q,N_k,3]
        nv = len(g.verts)
        Bv = np.zeros((nE, nv, 3))
        for c in range(3):
            Mc = (m1 * qw[:, None]).T @ gk[:, :, c]   # [4, N_k]
            Bv[:, :, c] = Pis.T @ Mc.T @ Pi1
        out["B"] = Bv.reshape(nE, nv * 3)
        # linear velocity data on the paper's scaled monomials (App. A)
        T = bs.linear_to_paper()
        out["Pi1s"] = T @ Pi1
        out["CPis"] = np.einsum("ij,cjk->cik", T, bs.deriv_to_linear(k)) @ Pis
        mp = mono3(qp, g.xc, g.hc, 1)
        out["M1"] = (mp * qw[:, None]).T @ mp
    return out


class StandaloneCell:
    """Cell geometry built directly from outward face polygons (for single-cell checks)."""

    def __init__(self, face_polys):
        pts = []
        faces = []
        for P in face_polys:
            cyc = []
            for p in P:
                for i, q in enumerate(pts):
                    if norm3(q - p) < 1e-12:
                        cyc.append(i)
                        break
                else:
                    pts.append(np.asarray(p, dtype=np.float64))
                    cyc.append(len(pts) - 1)
            faces.append(cyc)
        self.X = np.array(pts)
        self.faces = faces
        self.face_ids = list(range(len(faces)))
        self.verts = []
        self.edge_index = {}
        self.edges = []
        for cyc in faces:
            for i in range(len(cyc)):
                a, b = cyc[i], cyc[(i + 1) % len(cyc)]
                if a not in self.verts:
                    self.verts.append(a)
                key = (a, b) if a < b else (b, a)
                if key not in self.edge_index:
                    self.edge_index[key] = len(self.edges)
                    self.edges.append(len(self.edges))
        self.edge_pairs = [None] * len(self.edges)
        for key, e in self.edge_index.items():
            self.edge_pairs[e] = key
        self.vloc = {v: i for i, v in enumerate(self.verts)}
        self.eloc = {e: e for e in self.edges}
        from .geometry import poly_volume_centroid
        self.volume, self.xc = poly_volume_centroid([(self.X[c], None, None) for c in faces])
        V = self.X[self.verts]
        d = V[:, None, :] - V[None, :, :]
        self.hc = float(np.sqrt((d ** 2).sum(-1).max()))
        self.basis = Basis3(V, self.xc, self.hc)

    def n_local(self, k):
        if k == 1:
            return len(self.verts)
        return len(self.verts) + len(self.edges) + len(self.faces) + 1
