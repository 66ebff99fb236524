"""Convex polyhedra and the binary-space cut-cell construction (Sec. 5.1).

A convex polyhedron is a list of faces; a face is a tuple ``(P, n, d)`` with
vertices ``P`` [m,3] counter-clockwise seen from outside, outward unit
normal ``n`` and plane offset ``d`` (n.x = d on the face).

The construction follows the paper's steps:
1. associate each boundary triangle with the background cells it meets,
2. per cell, order the triangles by how many other triangles of that cell
   their supporting plane crosses (fewest first),
3. split the cell by each triangle's plane in that order, sending the
   remaining triangles to the sub-cells they meet, skipping cuts that would
   leave a part of volume below 1e-12,
4. classify every leaf as interior (solid) or exterior (fluid).

Readings taken where the paper is loose (each is a convention, parity
unpinned):
* association uses an exact triangle/box overlap test (a superset of any
  point sampling of the triangle);
* "crossing" means the plane leaves vertices of the other triangle strictly
  on both sides (tolerance 1e-12), ties broken by triangle index;
* a triangle is sent to a sub-cell when its clipped area there exceeds
  1e-14 h^2; triangles coplanar with the cut are consumed by it;
* interior/exterior is decided by the winding number of the closed boundary
  mesh at the leaf centroid (a ray cast; a leaf is never crossed by a
  triangle, so its centroid decides the whole leaf); interior when > 0.
"""
import math
import numpy as np

PLANE_TOL = 1e-12


def cross3(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def norm3(a):
    return math.sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2])


MIN_VOLUME = 1e-12


# --------------------------------------------------------------------------- polygons

def polygon_area_vec(P):
    """Vector area (1/2) sum_i p_i x p_{i+1}, with positions taken about p_0.

    The shift leaves the sum unchanged in exact arithmetic; in floating point
    it keeps a face much smaller than its distance from the origin from
    cancelling to zero.
    """
    R = P - P[0]
    Q = np.roll(R, -1, axis=0)
    return 0.5 * np.stack([R[:, 1] * Q[:, 2] - R[:, 2] * Q[:, 1],
                           R[:, 2] * Q[:, 0] - R[:, 0] * Q[:, 2],
                           R[:, 0] * Q[:, 1] - R[:, 1] * Q[:, 0]], -1).sum(0)


def polygon_area(P):
    return norm3(polygon_area_vec(P))


def clip_polygon(P, n, d, tol=PLANE_TOL):
    """Part of polygon P inside the half-space n.x <= d."""
    if len(P) == 0:
        return P
    s = P @ n - d
    out = []
    m = len(P)
    for i in range(m):
        a, b = P[i], P[(i + 1) % m]
        sa, sb = s[i], s[(i + 1) % m]
        if sa <= tol:
            out.append(a)
        if (sa < -tol and sb > tol) or (sa > tol and sb < -tol):
            out.append(_edge_plane_point(a, b, sa, sb))
    if len(out) < 3:
        return np.zeros((0, 3))
    return _dedupe_cycle(np.array(out))


def _edge_plane_point(a, b, sa, sb):
    # endpoint order fixed lexicographically so both orientations round alike
    if tuple(a) > tuple(b):
        a, b, sa, sb = b, a, sb, sa
    t = sa / (sa - sb)
    return a + t * (b - a)


def _dedupe_cycle(P, tol=1e-13):
    keep = []
    for i in range(len(P)):
        if not keep or norm3(P[i] - keep[-1]) > tol:
            keep.append(P[i])
    while len(keep) > 1 and norm3(keep[0] - keep[-1]) <= tol:
        keep.pop()
    return np.array(keep) if len(keep) >= 3 else np.zeros((0, 3))


def order_on_plane(points, n):
    """Sort coplanar points counter-clockwise around their mean seen along +n."""
    c = points.mean(axis=0)
    t1 = points[0] - c
    if np.linalg.norm(t1) < 1e-300:
        t1 = np.cross(n, [1.0, 0.0, 0.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    ang = np.arctan2((points - c) @ t2, (points - c) @ t1)
    return points[np.argsort(ang, kind="stable")]


def unique_points(points, tol=1e-13):
    out = []
    for p in points:
        if all(norm3(p - q) > tol for q in out):
            out.append(p)
    return np.array(out) if out else np.zeros((0, 3))


# --------------------------------------------------------------------------- polyhedra

def make_box(lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    c = lambda x, y, z: np.array([x, y, z], dtype=np.float64)
    faces = [
        (np.array([c(x0, y0, z0), c(x0, y0, z1), c(x0, y1, z1), c(x0, y1, z0)]), np.array([-1.0, 0, 0]), -x0),
        (np.array([c(x1, y0, z0), c(x1, y1, z0), c(x1, y1, z1), c(x1, y0, z1)]), np.array([1.0, 0, 0]), x1),
        (np.array([c(x0, y0, z0), c(x1, y0, z0), c(x1, y0, z1), c(x0, y0, z1)]), np.array([0, -1.0, 0]), -y0),
        (np.array([c(x0, y1, z0), c(x0, y1, z1), c(x1, y1, z1), c(x1, y1, z0)]), np.array([0, 1.0, 0]), y1),
        (np.array([c(x0, y0, z0), c(x0, y1, z0), c(x1, y1, z0), c(x1, y0, z0)]), np.array([0, 0, -1.0]), -z0),
        (np.array([c(x0, y0, z1), c(x1, y0, z1), c(x1, y1, z1), c(x0, y1, z1)]), np.array([0, 0, 1.0]), z1),
    ]
    return faces


def poly_volume_centroid(faces):
    """Volume and centroid from the (centre, face mean, edge) tetrahedra."""
    allp = np.concatenate([f[0] for f in faces])
    o = allp.mean(axis=0)
    A, B, C = [], [], []
    for f in faces:
        P = f[0]
        A.append(np.broadcast_to(P.mean(axis=0), P.shape))
        B.append(P)
        C.append(np.roll(P, -1, axis=0))
    A = np.concatenate(A) - o
    B = np.concatenate(B) - o
    C = np.concatenate(C) - o
    v = np.einsum("ij,ij->i", A, np.cross(B, C)) / 6.0
    vol = float(v.sum())
    cen = o + (v[:, None] * (A + B + C)).sum(0) / (4.0 * vol) if vol != 0 else o
    return vol, cen


def poly_vertices(faces):
    return unique_points(np.concatenate([f[0] for f in faces]))


def split_polyhedron(faces, n, d, tol=PLANE_TOL):
    """Return (below, above): the parts of the polyhedron with n.x <= d and >= d.

    Either part is None when the plane does not cut the polyhedron.
    """
    allp = np.concatenate([f[0] for f in faces])
    s = allp @ n - d
    if s.max() <= tol:
        return faces, None
    if s.min() >= -tol:
        return None, faces
    below, above, cap = [], [], []
    for P, fn, fd in faces:
        sp = P @ n - d
        cap.extend(P[np.abs(sp) <= tol])
        m = len(P)
        for i in range(m):
            if (sp[i] < -tol and sp[(i + 1) % m] > tol) or (sp[i] > tol and sp[(i + 1) % m] < -tol):
                cap.append(_edge_plane_point(P[i], P[(i + 1) % m], sp[i], sp[(i + 1) % m]))
        lo = clip_polygon(P, n, d, tol)
        hi = clip_polygon(P, -n, -d, tol)
        if len(lo) >= 3 and polygon_area(lo) > 0:
            below.append((lo, fn, fd))
        if len(hi) >= 3 and polygon_area(hi) > 0:
            above.append((hi, fn, fd))
    cap = unique_points(np.array(cap))
    if len(cap) >= 3:
        below.append((order_on_plane(cap, n), n.copy(), d))
        above.append((order_on_plane(cap, -n), -n, -d))
    return below, above


def clip_polygon_to_poly(P, faces):
    """Part of polygon P inside the convex polyhedron."""
    for _, fn, fd in faces:
        P = clip_polygon(P, fn, fd)
        if len(P) < 3:
            return np.zeros((0, 3))
    return P


# --------------------------------------------------------------------------- triangles vs boxes

def tri_box_overlap(a, b, c, lo, hi, eps=1e-12):
    """Separating-axis test (Akenine-Moller) between a triangle and a closed box."""
    centre = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo) + eps
    v = [a - centre, b - centre, c - centre]
    e = [v[1] - v[0], v[2] - v[1], v[0] - v[2]]
    for i in range(3):
        lo_i = min(v[0][i], v[1][i], v[2][i])
        hi_i = max(v[0][i], v[1][i], v[2][i])
        if lo_i > half[i] or hi_i < -half[i]:
            return False
    n = cross3(e[0], e[1])
    r = float(half @ np.abs(n))
    if abs(float(n @ v[0])) > r:
        return False
    E = np.array(e)                                   # [3 edges, 3]
    Vv = np.array(v)                                  # [3 verts, 3]
    for i in range(3):
        ax = np.zeros((3, 3))
        ax[:, (i + 1) % 3] = -E[:, (i + 2) % 3]      # e_i x edge, for unit axis i
        ax[:, (i + 2) % 3] = E[:, (i + 1) % 3]
        p = ax @ Vv.T                                  # [edges, verts]
        r = np.abs(ax) @ half
        nz = (ax * ax).sum(1) > 1e-300
        if np.any(nz & ((p.min(1) > r) | (p.max(1) < -r))):
            return False
    return True


def associate_triangles(V, F, N):
    """Map background cell (i,j,k) -> sorted list of triangle indices meeting it."""
    h = 1.0 / N
    cells = {}
    for t, (ia, ib, ic) in enumerate(F):
        a, b, c = V[ia], V[ib], V[ic]
        lo = np.minimum(np.minimum(a, b), c)
        hi = np.maximum(np.maximum(a, b), c)
        i0 = np.clip(np.floor(lo / h - 1e-9).astype(int), 0, N - 1)
        i1 = np.clip(np.floor(hi / h + 1e-9).astype(int), 0, N - 1)
        for i in range(i0[0], i1[0] + 1):
            for j in range(i0[1], i1[1] + 1):
                for k in range(i0[2], i1[2] + 1):
                    blo = np.array([i, j, k]) * h
                    if tri_box_overlap(a, b, c, blo, blo + h):
                        cells.setdefault((i, j, k), []).append(t)
    return cells


# --------------------------------------------------------------------------- BSP

class Node:
    __slots__ = ("faces", "plane", "children", "weight", "parent", "fluid", "volume", "centroid", "id")

    def __init__(self, faces, parent, nid):
        self.faces = faces
        self.plane = None
        self.children = None
        self.weight = 0.0
        self.parent = parent
        self.fluid = None
        self.id = nid
        self.volume, self.centroid = poly_volume_centroid(faces)


def triangle_planes(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    area2 = np.linalg.norm(n, axis=1)
    n = n / area2[:, None]
    d = np.einsum("ij,ij->i", n, a)
    return n, d, 0.5 * area2


def build_cell_tree(bg, tris, V, F, planes, total_area, h):
    """Binary space partition of one background cell; returns the node list."""
    n_t, d_t, _ = planes
    lo = np.array(bg, dtype=np.float64) * h
    root = Node(make_box(lo, lo + h), -1, 0)
    nodes = [root]
    # order: fewest crossings of the supporting plane with the cell's other triangles
    counts = []
    for t in tris:
        cnt = 0
        for s in tris:
            if s == t:
                continue
            sd = V[F[s]] @ n_t[t] - d_t[t]
            if sd.max() > PLANE_TOL and sd.min() < -PLANE_TOL:
                cnt += 1
        counts.append(cnt)
    order = [t for _, t in sorted(zip(counts, tris))]
    area_tol = 1e-14 * h * h

    def tri_in(t, faces):
        P = clip_polygon_to_poly(V[F[t]], faces)
        return len(P) >= 3 and polygon_area(P) > area_tol

    stack = [(0, order)]
    while stack:
        nid, pending = stack.pop()
        node = nodes[nid]
        while pending:
            t = pending[0]
            rest = pending[1:]
            coplanar = [s for s in pending
                        if np.all(np.abs(V[F[s]] @ n_t[t] - d_t[t]) <= PLANE_TOL)]
            below, above = split_polyhedron(node.faces, n_t[t], d_t[t])
            if below is None or above is None:
                pending = [s for s in rest if s not in coplanar]
                continue
            vb, _ = poly_volume_centroid(below)
            va, _ = poly_volume_centroid(above)
            if vb < MIN_VOLUME or va < MIN_VOLUME:
                pending = [s for s in rest if s not in coplanar]
                continue
            # importance weight: boundary-covered part of the cut polygon / total area
            covered = 0.0
            for s in coplanar:
                P = clip_polygon_to_poly(V[F[s]], node.faces)
                if len(P) >= 3:
                    covered += polygon_area(P)
            node.plane = (n_t[t].copy(), float(d_t[t]))
            node.weight = covered / total_area
            rest = [s for s in rest if s not in coplanar]
            kids = []
            for part in (below, above):
                child = Node(part, nid, len(nodes))
                nodes.append(child)
                kids.append(child.id)
                stack.append((child.id, [s for s in rest if tri_in(s, part)]))
            node.children = tuple(kids)
            break
    return nodes


# --------------------------------------------------------------------------- classification

RAY_DIR = np.array([3.1e-5 * np.sqrt(2.0), 1.7e-5 * np.sqrt(3.0), 1.0])
RAY_DIR = RAY_DIR / np.linalg.norm(RAY_DIR)


class InsideTest:
    """Winding number of a closed outward mesh along a slightly tilted +z ray."""

    def __init__(self, V, F, N):
        self.V, self.F, self.N = V, F, N
        a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
        self.a, self.e1, self.e2 = a, b - a, c - a
        self.n = np.cross(self.e1, self.e2)
        lo = np.minimum(np.minimum(a, b), c)
        hi = np.maximum(np.maximum(a, b), c)
        h = 1.0 / N
        self.cols = {}
        pad = 1e-3 * h + 1e-4
        i0 = np.clip(np.floor((lo[:, 0] - pad) / h).astype(int), 0, N - 1)
        i1 = np.clip(np.floor((hi[:, 0] + pad) / h).astype(int), 0, N - 1)
        j0 = np.clip(np.floor((lo[:, 1] - pad) / h).astype(int), 0, N - 1)
        j1 = np.clip(np.floor((hi[:, 1] + pad) / h).astype(int), 0, N - 1)
        for t in range(len(F)):
            for i in range(i0[t], i1[t] + 1):
                for j in range(j0[t], j1[t] + 1):
                    self.cols.setdefault((i, j), []).append(t)
        self.cols = {k: np.array(v) for k, v in self.cols.items()}

    def winding(self, p):
        h = 1.0 / self.N
        key = (min(int(p[0] / h), self.N - 1), min(int(p[1] / h), self.N - 1))
        ts = self.cols.get(key)
        if ts is None:
            return 0
        d = RAY_DIR
        e1, e2, a = self.e1[ts], self.e2[ts], self.a[ts]
        pv = np.cross(d, e2)
        det = np.einsum("ij,ij->i", e1, pv)
        ok = np.abs(det) > 1e-300
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        tv = p - a
        u = np.einsum("ij,ij->i", tv, pv) * inv
        qv = np.cross(tv, e1)
        v = (qv @ d) * inv
        t = np.einsum("ij,ij->i", e2, qv) * inv
        hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        sgn = np.sign(self.n[ts] @ d)
        return int(np.sum(sgn[hit]))

    def inside(self, p):
        return self.winding(p) > 0
