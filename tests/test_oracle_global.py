"""Pins of the oracle's grid, hierarchy, transfers and solver.

Checks are invariants and exact identities the paper or the mathematics fix:
convex cut cells tiling each background cell (Sec. 5.1), nestedness
(Sec. 5.2), exact reproduction of polynomial pressures (patch test,
Sec. 3.1), polynomial reproduction of the prolongation (Sec. 4), the
diffusion-free coupling pattern of A_c (Sec. 4), the Galerkin identity by
dense brute force, the Chebyshev error polynomial (textbook closed form),
V-cycle symmetry, PCG against a sparse direct solve, and the adjoint
dot-product identity.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.multigrid import chebyshev, galerkin
from oracle.quadrature import polygon_rule, polyhedron_rule
from oracle.vem import mono3


def _dof_values(pb, level, q):
    """DOF vector (free DOFs of the level) of a global polynomial q."""
    m, d = pb.meshes[level], pb.dofs[level]
    X = m.X
    vals = [q(X)]
    if d.k == 2:
        vals.append(q(0.5 * (X[m.edges[:, 0]] + X[m.edges[:, 1]])))
        fm = []
        for f in m.faces:
            qp, qw = polygon_rule(X[f])
            fm.append(qw @ q(qp) / qw.sum())
        vals.append(np.array(fm))
        cm = []
        for c in range(len(m.cell_faces)):
            from oracle.vem import CellGeometry
            g = CellGeometry(m, c)
            qp, qw = polyhedron_rule([X[cyc] for cyc in g.faces])
            cm.append(qw @ q(qp) / qw.sum())
        vals.append(np.array(cm))
    full = np.concatenate(vals)
    return full[d.free_ids]


def _poly(k, seed):
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal(10 if k == 2 else 4)
    xc = np.array([0.5, 0.5, 0.5])

    def q(X):
        return mono3(np.atleast_2d(X), xc, 1.0, k) @ coef

    def grad(X):
        from oracle.vem import grad_mono3
        return np.einsum("qic,i->qc", grad_mono3(np.atleast_2d(X), xc, 1.0, k), coef)
    return q, grad


# ------------------------------------------------------------------ grid invariants

@pytest.mark.parametrize("fx", ["c1_small", "c3_small", "c4_small"])
def test_cells_convex_and_closed(fx, request):
    pb = request.getfixturevalue(fx)
    m = pb.meshes[0]
    for c in range(len(m.cell_faces)):
        nv, ne, nf = len(m.cell_verts[c]), len(m.cell_edges[c]), len(m.cell_face_ids[c])
        assert nv - ne + nf == 2
        assert m.cell_volume[c] >= 1e-12
        Xc = m.X[m.cell_verts[c]]
        for f, o in m.cell_faces[c]:
            n = m.face_normal[f] * o
            d = n @ m.X[m.faces[f][0]]
            # vertices are merged within 2e-10; on the 1e-5-thin sliver faces
            # of the sheet that tilts the fitted face normal by up to ~1e-7
            assert (Xc @ n - d).max() < 1e-7
    assert all(1 <= len(fc) <= 2 for fc in m.face_cells)


@pytest.mark.parametrize("fx", ["c1_small", "c3_small", "c4_small"])
def test_leaves_tile_background_cells(fx, request):
    pb = request.getfixturevalue(fx)
    h = pb.forest.h
    for bg, nodes in pb.forest.trees.items():
        vol = sum(nd.volume for nd in nodes if nd.children is None)
        assert abs(vol - h ** 3) < 1e-12 * h ** 3 + 1e-15
        for nd in nodes:
            if nd.children is None:
                assert nd.volume >= 1e-12


@pytest.mark.parametrize("fx", ["c1_small", "c3_small"])
def test_hierarchy_nested(fx, request):
    pb = request.getfixturevalue(fx)
    for t, par in enumerate(pb.parents):
        mf, mc = pb.meshes[t], pb.meshes[t + 1]
        assert len(par) == len(mf.cell_faces)
        for c, E in enumerate(par):
            Xf = mf.X[mf.cell_verts[c]]
            for f, o in mc.cell_faces[E]:
                n = mc.face_normal[f] * o
                d = n @ mc.X[mc.faces[f][0]]
                assert (Xf @ n - d).max() < 1e-7
        # every coarse cell holds at least one fine cell
        assert len(set(par.tolist())) == len(mc.cell_faces)


# ------------------------------------------------------------------ operators

@pytest.mark.parametrize("fx", ["c1_small", "c2_small", "c3_small"])
def test_K_symmetric_and_null_space(fx, request):
    pb = request.getfixturevalue(fx)
    K = pb.K
    assert abs(K - K.T).max() < 1e-12 * abs(K).max()
    if pb.w.dirichlet_top:
        np.linalg.cholesky(K.toarray())          # SPD with p = 0 on the top face
        assert len(pb.null.floating) == 0
    else:
        assert np.abs(K @ np.ones(K.shape[0])).max() < 1e-11 * abs(K).max()
        assert len(pb.null.floating) >= 1


@pytest.mark.parametrize("fx", ["c2_small", "c3_small", "c4_small"])
def test_global_patch_test(fx, request):
    """u = grad q for q in P_k: K D(q) = B u exactly and the solve returns D(q) + const."""
    pb = request.getfixturevalue(fx)
    q, grad = _poly(pb.k, 3)
    Dq = _dof_values(pb, 0, q)
    u = grad(pb.vertices).ravel()
    lhs = pb.K @ Dq
    rhs = pb.B @ u
    # per-row backward error: 1e-5-thin cells have |K| entries ~1e3 whose
    # products cancel to O(1e-2), so an absolute bound would be meaningless
    scale = abs(pb.K) @ np.abs(Dq) + abs(pb.B) @ np.abs(u)
    assert (np.abs(lhs - rhs) / scale).max() < 1e-11
    p = pb.solve_direct(u)
    ref = pb.null.project(Dq)
    assert np.linalg.norm(p - ref) < 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("fx", ["c1_small", "c3_small", "c4_small"])
def test_prolongation_reproduces_polynomials(fx, request):
    pb = request.getfixturevalue(fx)
    q, _ = _poly(pb.k, 5)
    if pb.w.dirichlet_top:
        # polynomials of order k vanishing on z = 1
        if pb.k == 1:
            q = lambda X: 0.7 * (1.0 - np.atleast_2d(X)[:, 2])
        else:
            q1, _ = _poly(1, 5)
            q = lambda X: (1.0 - np.atleast_2d(X)[:, 2]) * q1(X)
    for t, P in enumerate(pb.P):
        Dc = _dof_values(pb, t + 1, q)
        Df = _dof_values(pb, t, q)
        # measured: 6e-16 (c1), 7e-15 (c3), 4e-13 (c4, whose 1e-5-thin cells
        # amplify rounding in their local projections)
        assert np.abs(P @ Dc - Df).max() < 1e-11 * max(np.abs(Df).max(), 1.0)


def test_prolongation_trilinear_on_uncut_grid():
    """No obstacle, k = 1, 2:1 aggregation: the prolongation is trilinear interpolation."""
    import synth
    from oracle.problem import Problem

    w = synth.get_config("c2", N=4, k=1, levels=2)
    w.mesh_fn = lambda N: (np.zeros((0, 3)), np.zeros((0, 3), dtype=np.int64))
    pb = Problem(w, coarse_max=0, max_levels=2)
    P = pb.P[0].toarray()
    Xf = pb.meshes[0].X[pb.dofs[0].free_ids]
    Xc = pb.meshes[1].X[pb.dofs[1].free_ids]
    H = 2.0 / 4
    W = np.prod(np.clip(1.0 - np.abs(Xf[:, None, :] - Xc[None, :, :]) / H, 0.0, None), axis=2)
    assert np.abs(P - W).max() < 1e-14


@pytest.mark.parametrize("fx", ["c1_small", "c3_small"])
def test_galerkin_brute_force_and_pattern(fx, request):
    pb = request.getfixturevalue(fx)
    A = pb.K
    for t, P in enumerate(pb.P[:2]):
        Ac = galerkin(A, P)
        Ad = P.toarray().T @ A.toarray() @ P.toarray()
        assert np.abs(Ac.toarray() - Ad).max() < 1e-12 * np.abs(Ad).max()
        assert abs(Ac - Ac.T).max() < 1e-12 * abs(Ac).max()
        # diffusion-free: A_c(i,j) != 0 only if i and j share a coarse cell
        d = pb.dofs[t + 1]
        allowed = set()
        for c in range(len(pb.meshes[t + 1].cell_faces)):
            ids = d.free[d.cell_dofs(c)]
            ids = ids[ids >= 0]
            for i in ids:
                for j in ids:
                    allowed.add((int(i), int(j)))
        coo = Ac.tocoo()
        big = np.abs(coo.data) > 1e-14 * np.abs(coo.data).max()
        assert all((int(i), int(j)) in allowed for i, j in zip(coo.row[big], coo.col[big]))
        A = Ac


def test_chebyshev_matches_closed_form():
    """With D^-1 A = diag(lam) the error is multiplied by T_5((th-lam)/de) / T_5(th/de)."""
    lam = np.linspace(0.01, 2.0, 40)
    dscale = np.linspace(0.5, 3.0, 40)
    A = sp.diags(lam * dscale).tocsr()          # D^-1 A = diag(lam) for D = diag(dscale)
    lmax = 2.0
    e0 = np.random.default_rng(0).standard_normal(40)
    b = A @ e0
    x = chebyshev(A, b, None, lmax, degree=5, lower=1.0 / 30.0, x_is_zero=True, dinv=1.0 / dscale)
    lo, hi = lmax / 30.0, lmax
    th, de = 0.5 * (hi + lo), 0.5 * (hi - lo)
    T5 = np.polynomial.chebyshev.Chebyshev([0, 0, 0, 0, 0, 1])
    ratio = T5((th - lam) / de) / T5(th / de)
    assert np.abs((e0 - x) - ratio * e0).max() < 1e-12


@pytest.mark.parametrize("fx", ["c1_small", "c3_small"])
def test_vcycle_symmetric_positive(fx, request, rng):
    pb = request.getfixturevalue(fx)
    n = pb.K.shape[0]
    x = pb.null.project(rng.standard_normal(n))
    y = pb.null.project(rng.standard_normal(n))
    Mx, My = pb.mg.vcycle(x), pb.mg.vcycle(y)
    assert abs(x @ My - y @ Mx) < 1e-10 * abs(x @ Mx)
    assert x @ Mx > 0 and y @ My > 0


@pytest.mark.parametrize("fx", ["c1_small", "c2_small", "c3_small", "c4_small"])
def test_mgpcg_matches_direct(fx, request):
    pb = request.getfixturevalue(fx)
    import synth
    u = synth.normal_field(pb.vertices, 0)
    p_ref = pb.solve_direct(u)
    p, it, hist = pb.solve_mgpcg(u, tol=1e-10)
    r = pb.rhs(u) - pb.K @ p
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(pb.rhs(u))
    assert np.linalg.norm(p - p_ref) <= 1e-7 * np.linalg.norm(p_ref)


@pytest.mark.parametrize("fx", ["c2_small", "c3_small"])
def test_adjoint_dot_product(fx, request, rng):
    pb = request.getfixturevalue(fx)
    u = rng.standard_normal(3 * pb.n_vertices)
    g = rng.standard_normal(pb.K.shape[0])
    p = pb.solve_direct(u)
    gu = pb.adjoint_direct(g)
    assert abs(p @ g - u @ gu) < 1e-10 * np.linalg.norm(p) * np.linalg.norm(g)
