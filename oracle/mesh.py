"""Conforming polyhedral mesh of the fluid cells of a convex tiling.

The paper obtains a conforming body-fitted grid from exact arithmetic (CGAL)
without describing the face bookkeeping.  Reading taken here: the whole unit
cube is tiled by convex cells (fluid and solid); the faces of a fluid cell are
the non-empty overlaps of its facets with the coplanar, opposite facets of its
neighbours (every overlap of two convex polygons is convex); coincident
vertices are merged within 1e-10 (the same intersection reached through
different clipping sequences differs by ~1e-12 where nearly parallel planes
meet, while distinct vertices of the paper's scenes stay above 1e-9 apart at
the grid sizes used); every vertex lying inside an edge of a face
is inserted into that face (T-junctions), so each shared face and edge is the
same polygon and segment on both sides.  Only fluid cells carry degrees of
freedom.
"""
import numpy as np

from .geometry import clip_polygon, polygon_area, polygon_area_vec, poly_volume_centroid, cross3, norm3

VERT_TOL = 1e-10
PLANE_MATCH = 1e-9


class Tile:
    """One convex cell of a tiling of the unit cube."""
    __slots__ = ("faces", "fluid", "lo", "hi", "cube_size", "key")

    def __init__(self, faces, fluid, lo, hi, cube_size, key):
        self.faces = faces          # list of (P, n, d)
        self.fluid = fluid
        self.lo = lo                # background-cell footprint [lo, hi)
        self.hi = hi
        self.cube_size = cube_size  # edge length in background cells, 0 if not a cube
        self.key = key


class Mesh:
    """Conforming mesh of fluid cells.

    X: [nv,3] vertices; faces: list of vertex-id cycles (stored orientation);
    face_normal: [nf,3] unit normals of the stored orientation; edges: [ne,2];
    cell_faces: per cell list of (face id, +1/-1 orientation w.r.t. outward).
    """

    def __init__(self):
        self.X = None
        self.faces = []
        self.face_normal = []
        self.face_cells = []
        self.edges = None
        self.cell_faces = []
        self.cell_tiles = []


class _VertexPool:
    def __init__(self, h):
        self.h = h
        self.X = []
        self.lattice = {}
        self.buckets = {}
        self.q = 1e-10

    def get(self, p):
        g = p / self.h
        r = np.rint(g)
        if np.all(np.abs(g - r) * self.h < VERT_TOL):
            key = (int(r[0]), int(r[1]), int(r[2]))
            vid = self.lattice.get(key)
            if vid is None:
                vid = len(self.X)
                self.X.append(r * self.h)
                self.lattice[key] = vid
            return vid
        b = np.floor(p / self.q).astype(np.int64)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for vid in self.buckets.get((b[0] + dx, b[1] + dy, b[2] + dz), ()):
                        if norm3(self.X[vid] - p) < VERT_TOL:
                            return vid
        vid = len(self.X)
        self.X.append(p.copy())
        self.buckets.setdefault((b[0], b[1], b[2]), []).append(vid)
        return vid


def _clip_by_polygon(P, Q, m):
    """Overlap of coplanar convex polygons P and Q (Q counter-clockwise about m)."""
    for i in range(len(Q)):
        a, b = Q[i], Q[(i + 1) % len(Q)]
        on = cross3(b - a, m)
        nn = norm3(on)
        if nn == 0:
            continue
        on /= nn
        P = clip_polygon(P, on, float(on @ a))
        if len(P) < 3:
            return P
    return P


def _width_ok(P):
    if len(P) < 3:
        return False
    A = polygon_area(P)
    per = float(np.linalg.norm(np.roll(P, -1, axis=0) - P, axis=1).sum())
    return per > 0 and 2.0 * A / per > 1e-11


def conform(tiles, N):
    h = 1.0 / N
    bgmap = {}
    for ti, t in enumerate(tiles):
        for i in range(t.lo[0], t.hi[0]):
            for j in range(t.lo[1], t.hi[1]):
                for k in range(t.lo[2], t.hi[2]):
                    bgmap.setdefault((i, j, k), []).append(ti)

    def shell(t):
        out = set()
        for i in range(max(t.lo[0] - 1, 0), min(t.hi[0] + 1, N)):
            for j in range(max(t.lo[1] - 1, 0), min(t.hi[1] + 1, N)):
                for k in range(max(t.lo[2] - 1, 0), min(t.hi[2] + 1, N)):
                    out.update(bgmap[(i, j, k)])
        return out

    def is_plain(ti, t, neigh):
        if not t.cube_size:
            return False
        return all(tiles[g].cube_size == t.cube_size for g in neigh)

    pool = _VertexPool(h)
    fluid = [ti for ti, t in enumerate(tiles) if t.fluid]
    cell_cycles = []   # per fluid cell: list of vertex-id cycles (outward)
    plain_flags = []
    for ti in fluid:
        t = tiles[ti]
        neigh = shell(t)
        neigh.discard(ti)
        plain = is_plain(ti, t, neigh)
        plain_flags.append(plain)
        pieces = []
        if plain:
            pieces = [(P, n) for P, n, d in t.faces]
        else:
            cand = [(g, Q, m, e) for g in sorted(neigh) for (Q, m, e) in tiles[g].faces]
            cn = np.array([c[2] for c in cand]).reshape(-1, 3)
            ce = np.array([c[3] for c in cand])
            for P, n, d in t.faces:
                got = []
                hit = np.nonzero((np.abs(cn + n).sum(1) < PLANE_MATCH) & (np.abs(ce + d) < PLANE_MATCH))[0]
                for ci in hit:
                    g, Q, m, e = cand[ci]
                    O = _clip_by_polygon(P, Q, m)
                    if _width_ok(O):
                        got.append(O)
                if not got:
                    got = [P]   # on the boundary of the unit cube
                else:
                    a_sum = sum(polygon_area(O) for O in got)
                    a_p = polygon_area(P)
                    if abs(a_sum - a_p) > 1e-9 * max(a_p, h * h):
                        raise RuntimeError(f"facet overlay does not cover the facet ({a_sum} vs {a_p})")
                pieces += [(O, n) for O in got]
        cycles = []
        for P, n in pieces:
            ids = []
            for p in P:
                v = pool.get(p)
                if not ids or ids[-1] != v:
                    ids.append(v)
            while len(ids) > 1 and ids[0] == ids[-1]:
                ids.pop()
            if len(ids) >= 3:
                cycles.append(ids)
        cell_cycles.append(cycles)

    X = np.array(pool.X)
    # T-junctions: insert every vertex lying strictly inside a face edge
    hb = 0.5 * h
    bucket = {}
    for vid, p in enumerate(X):
        bucket.setdefault(tuple(np.floor(p / hb).astype(int)), []).append(vid)

    def on_segment(a, b):
        pa, pb = X[a], X[b]
        lo = np.floor((np.minimum(pa, pb) - 1e-9) / hb).astype(int)
        hi = np.floor((np.maximum(pa, pb) + 1e-9) / hb).astype(int)
        ab = pb - pa
        L2 = ab @ ab
        found = []
        for i in range(lo[0], hi[0] + 1):
            for j in range(lo[1], hi[1] + 1):
                for k in range(lo[2], hi[2] + 1):
                    for v in bucket.get((i, j, k), ()):
                        if v == a or v == b:
                            continue
                        w = X[v] - pa
                        tau = (w @ ab) / L2
                        if tau <= 1e-12 or tau >= 1 - 1e-12:
                            continue
                        if norm3(w - tau * ab) < VERT_TOL:
                            found.append((tau, v))
        found.sort()
        return [v for _, v in found]

    for ci, cycles in enumerate(cell_cycles):
        if plain_flags[ci]:
            continue
        out = []
        for cyc in cycles:
            new = []
            for i in range(len(cyc)):
                a, b = cyc[i], cyc[(i + 1) % len(cyc)]
                new.append(a)
                new += on_segment(a, b)
            out.append(new)
        cell_cycles[ci] = out

    mesh = Mesh()
    mesh.X = X
    face_index = {}
    edge_index = {}
    edges = []
    for ci, cycles in enumerate(cell_cycles):
        cf = []
        for cyc in cycles:
            key = tuple(sorted(cyc))
            P = X[cyc]
            nvec = polygon_area_vec(P)
            nvec /= norm3(nvec)
            fid = face_index.get(key)
            if fid is None:
                fid = len(mesh.faces)
                face_index[key] = fid
                mesh.faces.append(list(cyc))
                mesh.face_normal.append(nvec)
                mesh.face_cells.append([ci])
                for i in range(len(cyc)):
                    a, b = cyc[i], cyc[(i + 1) % len(cyc)]
                    ek = (a, b) if a < b else (b, a)
                    if ek not in edge_index:
                        edge_index[ek] = len(edges)
                        edges.append(ek)
                cf.append((fid, 1))
            else:
                mesh.face_cells[fid].append(ci)
                if len(mesh.face_cells[fid]) > 2:
                    raise RuntimeError("face shared by more than two cells")
                cf.append((fid, 1 if mesh.face_normal[fid] @ nvec > 0 else -1))
        mesh.cell_faces.append(cf)
    mesh.face_normal = np.array(mesh.face_normal)
    mesh.edges = np.array(edges, dtype=np.int64).reshape(-1, 2)
    mesh.edge_index = edge_index
    mesh.cell_tiles = fluid
    mesh.h = h
    mesh.N = N
    _cell_topology(mesh)
    return mesh


def _cell_topology(mesh):
    """Per cell: ordered vertex ids, edge ids, face ids, volume and centroid."""
    mesh.cell_verts, mesh.cell_edges, mesh.cell_face_ids = [], [], []
    mesh.cell_volume, mesh.cell_centroid = [], []
    for cf in mesh.cell_faces:
        verts, edges, fids = [], [], []
        seen_v, seen_e = set(), set()
        faces_geo = []
        for fid, o in cf:
            cyc = mesh.faces[fid] if o > 0 else mesh.faces[fid][::-1]
            fids.append(fid)
            for i in range(len(cyc)):
                a, b = cyc[i], cyc[(i + 1) % len(cyc)]
                if a not in seen_v:
                    seen_v.add(a)
                    verts.append(a)
                ek = (a, b) if a < b else (b, a)
                e = mesh.edge_index[ek]
                if e not in seen_e:
                    seen_e.add(e)
                    edges.append(e)
            P = mesh.X[cyc]
            faces_geo.append((P, None, None))
        vol, cen = poly_volume_centroid(faces_geo)
        mesh.cell_verts.append(verts)
        mesh.cell_edges.append(edges)
        mesh.cell_face_ids.append(fids)
        mesh.cell_volume.append(vol)
        mesh.cell_centroid.append(cen)
    mesh.cell_volume = np.array(mesh.cell_volume)
    mesh.cell_centroid = np.array(mesh.cell_centroid)


def cell_faces_outward(mesh, c):
    """Vertex-id cycles of cell c's faces, counter-clockwise seen from outside."""
    return [mesh.faces[f] if o > 0 else mesh.faces[f][::-1] for f, o in mesh.cell_faces[c]]
