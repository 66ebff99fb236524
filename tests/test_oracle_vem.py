"""Pins of the oracle's virtual-element operators against closed forms and exact identities.

Every check here is independent of the oracle's own formulas: a textbook
special case (P1 FEM on a tetrahedron), a hand-derived closed form (the k = 1
cube), exactness identities of projections (a projector reproduces
polynomials) and the VEM patch test (exact reproduction of polynomial
pressures of the method's order, Sec. 3.1).
"""
import numpy as np
import pytest

from oracle.geometry import make_box, split_polyhedron
from oracle.quadrature import polygon_rule, polyhedron_rule
from oracle.vem import (StandaloneCell, cell_projector, element_matrices, face_projector,
                        mono3, EXP3)


def _tet_faces(V):
    a, b, c, d = V
    faces = [[a, c, b], [a, b, d], [a, d, c], [b, c, d]]
    out = []
    cen = V.mean(axis=0)
    for f in faces:
        f = np.array(f)
        n = np.cross(f[1] - f[0], f[2] - f[0])
        if n @ (f[0] - cen) < 0:
            f = f[::-1]
        out.append(f)
    return out


def _cut_cell():
    """A genuinely polyhedral convex cell: a cube clipped by an oblique plane."""
    faces = make_box([0.1, 0.2, 0.3], [0.35, 0.45, 0.55])
    n = np.array([0.3, -0.5, 0.8])
    n /= np.linalg.norm(n)
    below, _ = split_polyhedron(faces, n, float(n @ np.array([0.25, 0.3, 0.42])))
    return StandaloneCell([f[0] for f in below])


def test_quadrature_exact_on_unit_cube_and_tet():
    faces = [f[0] for f in make_box([0, 0, 0], [1, 1, 1])]
    qp, qw = polyhedron_rule(faces)
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                exact = 1.0 / ((a + 1) * (b + 1) * (c + 1))
                assert abs(qw @ (qp[:, 0] ** a * qp[:, 1] ** b * qp[:, 2] ** c) - exact) < 1e-14
    # unit simplex: int x^a y^b z^c = a! b! c! / (a+b+c+3)!
    from math import factorial
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    qp, qw = polyhedron_rule(_tet_faces(V))
    for a, b, c in [(0, 0, 0), (1, 0, 0), (2, 1, 0), (1, 1, 1), (3, 0, 1), (2, 2, 0)]:
        exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        assert abs(qw @ (qp[:, 0] ** a * qp[:, 1] ** b * qp[:, 2] ** c) - exact) < 1e-15
    # polygon: unit square x^a y^b
    P = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0.0]])
    qp, qw = polygon_rule(P)
    assert abs(qw @ (qp[:, 0] ** 3 * qp[:, 1] ** 2) - 1.0 / 12.0) < 1e-15


@pytest.mark.parametrize("k", [1, 2])
def test_projector_reproduces_polynomials(k):
    g = _cut_cell()
    Pis, D, G = cell_projector(g, k)
    assert np.abs(Pis @ D - np.eye(len(Pis))).max() < 1e-11
    # face projections reproduce face polynomials
    for cyc in g.faces:
        P = g.X[cyc]
        n = np.cross(P[1] - P[0], P[2] - P[0])
        n /= np.linalg.norm(n)
        Pif, fr = face_projector(P, n, k)
        m = len(P)
        Df = [fr.mono(P, k)]
        if k == 2:
            Df.append(fr.mono(0.5 * (P + np.roll(P, -1, axis=0)), k))
            qp, qw = polygon_rule(P)
            Df.append((qw @ fr.mono(qp, k) / qw.sum())[None, :])
        Df = np.concatenate(Df)
        assert np.abs(Pif @ Df - np.eye(len(Pif))).max() < 1e-11


def test_k1_tetrahedron_equals_p1_fem():
    """V_1 on a tetrahedron is P_1, the stabilisation vanishes: K is the P1 FEM stiffness."""
    V = np.array([[0.1, 0.0, 0.2], [0.5, 0.1, 0.1], [0.2, 0.6, 0.0], [0.25, 0.2, 0.7]])
    g = StandaloneCell(_tet_faces(V))
    em = element_matrices(g, 1, with_velocity=False)
    X = g.X[g.verts]
    M = np.hstack([np.ones((4, 1)), X])
    grads = np.linalg.inv(M)[1:, :].T          # rows: gradient of barycentric lambda_i
    vol = abs(np.linalg.det(M)) / 6.0
    Kfem = vol * grads @ grads.T
    assert np.abs(em["K"] - Kfem).max() < 1e-13 * np.abs(Kfem).max()


def test_k1_cube_closed_form():
    """Cube of side h: consistency h s_i.s_j/16, projector (11^T + S S^T)/8."""
    h = 0.125
    g = StandaloneCell([f[0] for f in make_box([0.5, 0.25, 0.0], [0.5 + h, 0.25 + h, h])])
    em = element_matrices(g, 1, with_velocity=False)
    X = g.X[g.verts]
    s = np.sign(X - X.mean(axis=0))
    Pi = (np.ones((8, 8)) + s @ s.T) / 8.0
    K = h * (s @ s.T) / 16.0 + np.sqrt(3.0) * h * (np.eye(8) - Pi).T @ (np.eye(8) - Pi)
    assert np.abs(em["K"] - K).max() < 1e-15


@pytest.mark.parametrize("k", [1, 2])
def test_element_matrix_symmetric_psd_and_kills_constants(k):
    g = _cut_cell()
    em = element_matrices(g, k)
    K = em["K"]
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    assert np.linalg.eigvalsh(K)[0] > -1e-12 * np.abs(K).max()
    assert np.abs(K @ np.ones(len(K))).max() < 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("k", [1, 2])
def test_local_patch_test(k):
    """For q in P_k and u = grad q (linear), K^E D(q) = B^E u on one cut cell."""
    g = _cut_cell()
    em = element_matrices(g, k)
    rng = np.random.default_rng(7)
    coef = rng.standard_normal(10 if k == 2 else 4)
    xc, hc = g.xc, g.hc

    def q(X):
        return mono3(X, xc, hc, k) @ coef

    def grad_q(X):
        from oracle.vem import grad_mono3
        return np.einsum("qic,i->qc", grad_mono3(X, xc, hc, k), coef)

    Dq = [q(g.X[g.verts])]
    if k == 2:
        Dq.append(q(np.array([0.5 * (g.X[a] + g.X[b]) for a, b in g.edge_pairs])))
        for cyc in g.faces:
            qp, qw = polygon_rule(g.X[cyc])
            Dq.append(np.array([qw @ q(qp) / qw.sum()]))
        qp, qw = polyhedron_rule([g.X[c] for c in g.faces])
        Dq.append(np.array([qw @ q(qp) / qw.sum()]))
    Dq = np.concatenate(Dq)
    u = grad_q(g.X[g.verts]).ravel()
    lhs = em["K"] @ Dq
    rhs = em["B"] @ u
    assert np.abs(lhs - rhs).max() < 1e-12 * max(np.abs(rhs).max(), 1e-30)


def test_monomial_order_matches_appendix():
    assert EXP3[:4] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_vector_area_of_a_tiny_face_far_from_the_origin():
    """A right triangle with legs 2^-30 near (0.82, 0.45, 0.59): its vector area is
    exactly 2^-61 along +z (every coordinate and the result are representable), which
    a sum of cross products of absolute positions loses to cancellation."""
    from oracle.geometry import polygon_area_vec
    o = np.array([0.8203125, 0.453125, 0.5859375])
    L = 2.0 ** -30
    P = np.array([o, o + [L, 0.0, 0.0], o + [0.0, L, 0.0]])
    a = polygon_area_vec(P)
    assert a[2] == 0.5 * L * L and a[0] == 0.0 and a[1] == 0.0


def test_element_of_a_cell_with_a_tiny_corner_face():
    """A 1/128 cube near (0.82, 0.82, 0.82) with a corner cut 2e-9 deep along (1,1,1).

    The cut face is an equilateral triangle of area (sqrt(3)/2) l^2; the element stays
    finite, symmetric and positive semi-definite with the constants as its only null
    vector (Sec. 3.1)."""
    from oracle.geometry import polygon_area_vec
    lo, hi, ell = 0.8203125, 0.828125, 2e-9
    n = np.ones(3) / np.sqrt(3.0)
    below, _ = split_polyhedron(make_box([lo] * 3, [hi] * 3), n, float(n @ np.array([hi, hi, hi - ell])))
    g = StandaloneCell([f[0] for f in below])
    assert len(g.faces) == 7
    tiny = min(float(np.linalg.norm(polygon_area_vec(g.X[c]))) for c in g.faces)
    assert abs(tiny - 0.5 * np.sqrt(3.0) * ell ** 2) <= 1e-6 * tiny
    K = element_matrices(g, 2, with_velocity=False)["K"]
    assert np.isfinite(K).all()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    assert np.abs(K.sum(axis=1)).max() <= 1e-13 * np.abs(K).max()
    w = np.linalg.eigvalsh(0.5 * (K + K.T))
    # the next eigenvalue is 3.6e-4 of the largest for any cut depth (1e-6 down to
    # 2e-9): the tiny face adds no near-null mode
    assert w[0] >= -1e-13 * w[-1] and w[1] >= 1e-4 * w[-1]
