"""Closed, outward-oriented triangle meshes of the synthetic obstacles.

Each function returns ``(V, F)``: ``V`` float64 [nv, 3] vertex positions and
``F`` int64 [nt, 3] triangles whose right-hand normal points out of the solid.
These are the boundary meshes that the binary-space cut-cell construction
takes as input (the paper embeds a triangle mesh into a Cartesian grid).
"""
import numpy as np


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1)[:, None]
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return V, F


def _subdivide(V, F):
    """Split every triangle into four, projecting new points onto the unit sphere."""
    V = list(map(tuple, V))
    index = {}

    def mid(a, b):
        key = (a, b) if a < b else (b, a)
        if key not in index:
            p = (np.array(V[a]) + np.array(V[b])) * 0.5
            p /= np.linalg.norm(p)
            index[key] = len(V)
            V.append(tuple(p))
        return index[key]

    out = []
    for a, b, c in F:
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
    return np.array(V, dtype=np.float64), np.array(out, dtype=np.int64)


def _orient_outward(V, F, inside_point):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, (a + b + c) / 3.0 - inside_point) < 0
    F = F.copy()
    F[flip] = F[flip][:, [0, 2, 1]]
    return F


def _max_edge(V, F):
    e = np.concatenate([V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 1]], V[F[:, 0]] - V[F[:, 2]]])
    return float(np.max(np.linalg.norm(e, axis=1)))


def unit_icosphere(max_edge):
    """Unit icosphere subdivided until no edge is longer than ``max_edge``."""
    V, F = _icosahedron()
    while _max_edge(V, F) > max_edge:
        V, F = _subdivide(V, F)
    return V, F


def icosphere(center, radius, max_edge):
    V, F = unit_icosphere(max_edge / radius)
    V = np.asarray(center, dtype=np.float64) + radius * V
    return V, _orient_outward(V, F, np.asarray(center, dtype=np.float64))


def ellipsoid(center, semi_axes, rotation, max_edge):
    """x = c + R diag(a) y for y on the unit icosphere (orientation preserved)."""
    a = np.asarray(semi_axes, dtype=np.float64)
    V, F = unit_icosphere(max_edge / float(np.max(a)))
    R = np.asarray(rotation, dtype=np.float64)
    V = np.asarray(center, dtype=np.float64) + (V * a) @ R.T
    return V, _orient_outward(V, F, np.asarray(center, dtype=np.float64))


def rot_x(deg):
    t = np.deg2rad(deg)
    c, s = np.cos(t), np.sin(t)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_z(deg):
    t = np.deg2rad(deg)
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def quat_to_matrix(q):
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def box(center, size, rotation=None):
    """Rectangular box as 12 triangles (two per face)."""
    c = np.asarray(center, dtype=np.float64)
    hs = 0.5 * np.asarray(size, dtype=np.float64)
    R = np.eye(3) if rotation is None else np.asarray(rotation, dtype=np.float64)
    corners = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)],
                       dtype=np.float64)
    V = c + (corners * hs) @ R.T
    # corner index = (sx>0) + 2 (sy>0) + 4 (sz>0)
    quads = [[0, 2, 3, 1], [4, 5, 7, 6], [0, 1, 5, 4], [2, 6, 7, 3], [0, 4, 6, 2], [1, 3, 7, 5]]
    F = []
    for q in quads:
        F += [[q[0], q[1], q[2]], [q[0], q[2], q[3]]]
    F = np.array(F, dtype=np.int64)
    return V, _orient_outward(V, F, c)


def merge_meshes(meshes):
    Vs, Fs, off = [], [], 0
    for V, F in meshes:
        Vs.append(V)
        Fs.append(F + off)
        off += len(V)
    return np.concatenate(Vs), np.concatenate(Fs)


def plate_pair(gap, thickness=0.05, side=0.6, tilt_deg=17.0, mid=(0.5, 0.5, 0.5)):
    """Two parallel plates whose facing sides are ``gap`` apart.

    The mid-plane passes through ``mid`` with normal Rx(tilt) e_z.
    """
    R = rot_x(tilt_deg)
    n = R @ np.array([0.0, 0.0, 1.0])
    off = 0.5 * gap + 0.5 * thickness
    m = np.asarray(mid, dtype=np.float64)
    p1 = box(m + off * n, (side, side, thickness), R)
    p2 = box(m - off * n, (side, side, thickness), R)
    return merge_meshes([p1, p2])


def thin_sheet(spacing, thickness=1e-5, lo=0.1, hi=0.9, amp=0.1):
    """Closed thin shell around z = 0.5 + amp sin(2 pi x) cos(2 pi y).

    Top and bottom surfaces sit at +-thickness/2, triangulated on a grid of
    the given spacing over [lo, hi]^2, joined by rim strips.
    """
    m = max(1, int(np.ceil((hi - lo) / spacing - 1e-9)))
    s = np.linspace(lo, hi, m + 1)
    X, Y = np.meshgrid(s, s, indexing="ij")
    Z = 0.5 + amp * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    top = np.stack([X, Y, Z + 0.5 * thickness], -1).reshape(-1, 3)
    bot = np.stack([X, Y, Z - 0.5 * thickness], -1).reshape(-1, 3)
    V = np.concatenate([top, bot])
    nb = (m + 1) ** 2

    def vid(i, j, layer):
        return layer * nb + i * (m + 1) + j

    F = []
    for i in range(m):
        for j in range(m):
            a, b, c, d = vid(i, j, 0), vid(i + 1, j, 0), vid(i + 1, j + 1, 0), vid(i, j + 1, 0)
            F += [[a, b, c], [a, c, d]]          # top: +z facing
            a, b, c, d = vid(i, j, 1), vid(i + 1, j, 1), vid(i + 1, j + 1, 1), vid(i, j + 1, 1)
            F += [[a, c, b], [a, d, c]]          # bottom: -z facing
    ring = ([(i, 0) for i in range(m)] + [(m, j) for j in range(m)]
            + [(i, m) for i in range(m, 0, -1)] + [(0, j) for j in range(m, 0, -1)])
    for t in range(len(ring)):
        i0, j0 = ring[t]
        i1, j1 = ring[(t + 1) % len(ring)]
        a, b = vid(i0, j0, 0), vid(i1, j1, 0)
        c, d = vid(i1, j1, 1), vid(i0, j0, 1)
        F += [[a, d, c], [a, c, b]]
    F = np.array(F, dtype=np.int64)
    # orient rim strips outward (away from the sheet's footprint centre)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    rim = np.arange(len(F)) >= 4 * m * m
    out = cen[:, :2] - 0.5 * (lo + hi)
    flip = rim & (np.einsum("ij,ij->i", n[:, :2], out) < 0)
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def mesh_area(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum())


def signed_volume(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)
