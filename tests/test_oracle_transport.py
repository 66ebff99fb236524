"""Pins of the oracle's simulation-step transfers (Algorithm 1, Sec. 3.2-3.3).

Each check fixes a value by something other than the oracle's own code: the
kernel's closed form, hand-computed averages, linear fields that the cell
polynomials carry exactly, the closed form of the midpoint rule on a linear
field, and mirror images across known planes.
"""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import transport as T
from oracle.velocity import operators


def test_kernel_closed_form():
    q = np.array([0.0, 0.25, 0.5, 1.0, 2.0])
    assert np.array_equal(T.kernel(q), np.array([1.0, 0.421875, 0.125, 0.0, 0.0]))


def test_p2g_hand_computed_average():
    R = 0.1
    X = np.array([[0.5, 0.5, 0.5], [0.0, 0.0, 0.0]])
    # particles at distances 0.05 and 0.03 from the first point, one beyond R
    xp = np.array([[0.55, 0.5, 0.5], [0.5, 0.47, 0.5], [0.5, 0.5, 0.62]])
    fp = np.array([[2.0, 1.0], [-4.0, 3.0], [100.0, 100.0]])
    w1, w2 = (1 - 0.25) ** 3, (1 - 0.09) ** 3
    want = (np.array([2.0, 1.0]) * w1 + np.array([-4.0, 3.0]) * w2) / (w1 + w2)
    out = T.p2g(X, xp, fp, R)
    assert np.allclose(out[0], want, rtol=1e-14, atol=0)
    # no particle inside the support of the second point: the value 0
    assert np.array_equal(out[1], [0.0, 0.0])


def test_p2g_reproduces_constants(rng):
    X = rng.uniform(0.2, 0.8, size=(50, 3))
    xp = rng.uniform(0, 1, size=(2000, 3))
    out = T.p2g(X, xp, np.full((2000, 1), 3.25), 0.1)
    assert np.allclose(out, 3.25, rtol=1e-14, atol=0)


def test_buoyancy_closed_form():
    u = np.arange(6, dtype=np.float64)
    out = T.buoyancy(u, np.array([1.0, 0.5]), np.array([2.0, 0.0]), 0.3, 0.7, 0.5)
    assert np.array_equal(out, [0, 1, 2 + 0.5 * (-0.3 + 1.4), 3, 4, 5 + 0.5 * (-0.15)])


@pytest.fixture(scope="module")
def c1():
    pb = oracle_problem("c1", 8)
    return pb, T.Locator(pb)


def test_locator_centroids_obstacle_and_outside(c1):
    pb, loc = c1
    cen = pb.meshes[0].cell_centroid
    assert all(loc.cell_of(cen[c]) == c for c in range(len(cen)))
    assert loc.cell_of([0.5, 0.5, 0.5]) == -1          # the sphere's centre is solid
    assert loc.cell_of([0.5, 0.5, 1.2]) == -1          # outside the box


def test_linear_field_is_carried_exactly(c1, rng):
    """Pi_1 of a linear velocity is itself, so the cell polynomial evaluated
    anywhere in the cell returns the field (pins the monomial convention)."""
    pb, loc = c1
    a, B = rng.standard_normal(3), rng.standard_normal((3, 3))
    u = (pb.vertices @ B.T + a).ravel()
    s = operators(pb)["Pi"] @ u
    pts = rng.uniform(0, 1, size=(300, 3))
    n = 0
    for x in pts:
        c = loc.cell_of(x)
        if c >= 0:
            assert np.allclose(T.eval_field(pb, s, c, x), a + B @ x, rtol=0, atol=1e-12)
            n += 1
    assert n > 100


def test_g2p_flip_and_pic_limits(c1, rng):
    pb, loc = c1
    nc = len(pb.asm.cells)
    s_new, s_old = rng.standard_normal(12 * nc), rng.standard_normal(12 * nc)
    xp = rng.uniform(0, 1, size=(200, 3))
    up = rng.standard_normal((200, 3))
    ghost = np.array([loc.cell_of(x) < 0 for x in xp])
    same = T.g2p(pb, loc, xp, up, s_old, s_old, 1.0, ghost)
    assert np.array_equal(same, up)                      # pure FLIP, no increment
    pic = T.g2p(pb, loc, xp, up, s_new, s_old, 0.0, ghost)
    for p in range(200):
        if ghost[p]:
            assert np.array_equal(pic[p], up[p])          # ghosts are never updated
        else:
            c = loc.cell_of(xp[p])
            assert np.allclose(pic[p], T.eval_field(pb, s_new, c, xp[p]), rtol=0, atol=1e-14)


def test_midpoint_rule_on_a_linear_field(c1, rng):
    """For v = A x the midpoint rule gives x + dt A x + dt^2/2 A^2 x; points
    near the box corner stay far from the sphere."""
    pb, loc = c1
    A = 0.5 * rng.standard_normal((3, 3))
    u = (pb.vertices @ A.T).ravel()
    s = operators(pb)["Pi"] @ u
    xp = rng.uniform(0.03, 0.12, size=(40, 3))
    dt = 0.02
    x2, n = T.advect(pb, loc, np.zeros((0, 3, 3)), xp, s, dt, np.zeros(40, dtype=bool))
    assert n == 1
    want = xp + dt * xp @ A.T + 0.5 * dt * dt * xp @ (A @ A).T
    assert np.allclose(x2, want, rtol=0, atol=1e-14)


def test_reflection_at_a_wall_and_an_obstacle(c1):
    pb, loc = c1
    V, F = pb.boundary
    tri = np.asarray(V)[np.asarray(F)]
    # the wall x = 1: a mirror image
    out = T.resolve(loc, tri, np.array([0.9, 0.05, 0.05]), np.array([1.1, 0.05, 0.05]))
    assert np.allclose(out, [0.9, 0.05, 0.05], rtol=0, atol=1e-15)
    # the sphere (r = 0.3): the end point is mirrored in the plane of the
    # triangle the segment meets first
    a, b = np.array([0.5, 0.5, 0.1]), np.array([0.5, 0.5, 0.3])
    t, n = T._first_crossing(a, b, tri)
    q = a + t * (b - a)
    assert abs(np.linalg.norm(q - 0.5) - 0.3) < 0.01    # on the tessellated sphere
    out = T.resolve(loc, tri, a, b)
    assert np.allclose(out, b - 2 * ((b - q) @ n) * n, rtol=0, atol=1e-14)
    assert loc.cell_of(out) >= 0
