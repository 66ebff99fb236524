"""Exact polynomial quadrature on simplices, polygons and convex polyhedra.

Collapsed (Duffy) tensor Gauss-Legendre rules: with n points per direction a
triangle rule integrates degree <= 2n-2 exactly and a tetrahedron rule degree
<= 2n-3 (n = 4: degrees 6 and 5; the method needs degree <= 4).  Polygons are fanned from their vertex mean and polyhedra split into
(vertex mean, face vertex mean, edge) tetrahedra, valid because every cell of
the cut-cell grid is convex.
"""
import numpy as np

_N = 4
_x, _w = np.polynomial.legendre.leggauss(_N)
_x = 0.5 * (_x + 1.0)
_w = 0.5 * _w

# reference triangle {u>=0, v>=0, u+v<=1}: x = u, y = v (1-u), J = (1-u)
_U, _V = np.meshgrid(_x, _x, indexing="ij")
_WT = (_w[:, None] * _w[None, :]) * (1.0 - _U)
TRI_BARY = np.stack([1.0 - _U - _V * (1.0 - _U), _U, _V * (1.0 - _U)], -1).reshape(-1, 3)
TRI_W = (_WT.reshape(-1)) * 2.0  # weights sum to 1 (area fraction)

_U3, _V3, _W3 = np.meshgrid(_x, _x, _x, indexing="ij")
_J3 = (1.0 - _U3) ** 2 * (1.0 - _V3)
_WW = (_w[:, None, None] * _w[None, :, None] * _w[None, None, :]) * _J3
_X1 = _U3
_X2 = _V3 * (1.0 - _U3)
_X3 = _W3 * (1.0 - _U3) * (1.0 - _V3)
TET_BARY = np.stack([1.0 - _X1 - _X2 - _X3, _X1, _X2, _X3], -1).reshape(-1, 4)
TET_W = _WW.reshape(-1) * 6.0  # weights sum to 1 (volume fraction)


def triangle_rule(a, b, c):
    """Points [Q,3] and weights [Q] (summing to the area) for triangle abc."""
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    pts = TRI_BARY @ np.stack([a, b, c])
    return pts, TRI_W * area


def tet_rule(a, b, c, d):
    vol = abs(np.dot(b - a, np.cross(c - a, d - a))) / 6.0
    pts = TET_BARY @ np.stack([a, b, c, d])
    return pts, TET_W * vol


def _cross(a, b):
    return np.stack([a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1],
                     a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2],
                     a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]], -1)


def triangles_rule(A, B, C):
    """Rule over a batch of triangles (rows of A, B, C)."""
    area = 0.5 * np.sqrt((_cross(B - A, C - A) ** 2).sum(1))
    pts = (np.einsum("q,tk->tqk", TRI_BARY[:, 0], A) + np.einsum("q,tk->tqk", TRI_BARY[:, 1], B)
           + np.einsum("q,tk->tqk", TRI_BARY[:, 2], C))
    return pts.reshape(-1, 3), (area[:, None] * TRI_W[None, :]).reshape(-1)


def polygon_rule(P):
    """Rule over a convex planar polygon with vertices P [m,3] in cyclic order."""
    c = np.broadcast_to(P.mean(axis=0), P.shape)
    return triangles_rule(c, P, np.roll(P, -1, axis=0))


def polyhedron_rule(faces, centre=None):
    """Rule over a convex polyhedron given as a list of face vertex arrays."""
    if centre is None:
        centre = np.concatenate(faces).mean(axis=0)
    F = [np.broadcast_to(P.mean(axis=0), P.shape) for P in faces]
    A = np.concatenate(F)
    B = np.concatenate(faces)
    C = np.concatenate([np.roll(P, -1, axis=0) for P in faces])
    O = np.broadcast_to(centre, A.shape)
    vol = np.abs(np.einsum("ij,ij->i", A - O, _cross(B - O, C - O))) / 6.0
    pts = (np.einsum("q,tk->tqk", TET_BARY[:, 0], O) + np.einsum("q,tk->tqk", TET_BARY[:, 1], A)
           + np.einsum("q,tk->tqk", TET_BARY[:, 2], B) + np.einsum("q,tk->tqk", TET_BARY[:, 3], C))
    return pts.reshape(-1, 3), (vol[:, None] * TET_W[None, :]).reshape(-1)
