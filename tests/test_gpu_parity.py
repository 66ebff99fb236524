"""Parity of the HIP solver with the FP64 oracle, through the C ABI.

The library receives the oracle's grid, element matrices and prolongations,
so every comparison is on identical inputs:
* level-0 K (assembled on the library side) and the Galerkin coarse
  operators (element-wise P^T A P) against the oracle's sparse products;
* one FP64 V-cycle against the oracle's V-cycle (both projected to zero
  mean; the coarsest generalised inverses differ only on directions the
  prolongation annihilates or constants);
* FP64 and mixed solves against the oracle's sparse direct solve, with the
  true residual evaluated on the oracle's K and b;
* the divergence B, its transpose, and the adjoint solve;
* bitwise repeatability and the error paths.
Tolerances: one FP64 V-cycle 1e-8 (1e-6 on the thin sheet, see the test);
FP64 path true residual <= 1e-10 and pressure error <= 1e-8;
mixed path pressure error <= 1e-6 after refinement to 1e-10; adjoint
relative error <= 1e-8 (FP64) against the oracle's exact adjoint.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle_desc import describe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _hier(pb, **kw):
    from paper_2607_17725_amd import fvem
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    kw.setdefault("lattice_min_fraction", 1e-6)   # lattice stencil rows wherever a class qualifies
    return fvem.Hierarchy(describe(pb), **kw)


_H = {}


def hier_for(request, name):
    if name not in _H:
        pb = request.getfixturevalue(name)
        print(f"[gpu parity] building hierarchy for {name}", flush=True)
        _H[name] = (_hier(pb), pb)
    return _H[name]


# the 8^3 instances of every workload, and c1 at its named 16^3 with the plates and
# the thin sheet at 16^3 (k = 2: several lattice tiles, a stencil level and a ragged
# tail on every level)
CASES = ["c1_small", "c2_small", "c3_small", "c4_small", "c1_16", "c3_16", "c4_16"]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_operators_match_oracle(name, request):
    from paper_2607_17725_amd import fvem
    h, pb = hier_for(request, name)
    rp, ci, va = h.level_matrix(0)
    K = sp.csr_matrix((va, ci, rp), shape=pb.K.shape)
    assert abs(K - pb.K).max() <= 1e-13 * abs(pb.K).max()
    A = pb.K
    for l, P in enumerate(pb.P):
        A = (P.T @ A @ P).tocsr()
        rp, ci, va = h.level_matrix(l + 1)
        G = sp.csr_matrix((va, ci, rp), shape=A.shape)
        assert abs(G - A).max() <= 1e-12 * abs(A).max(), f"level {l + 1}"
    rng = np.random.default_rng(3)
    u = rng.standard_normal(3 * pb.n_vertices)
    g = rng.standard_normal(pb.K.shape[0])
    b = _host(h.apply(fvem.OP_B, _dev(u)))
    assert np.abs(b - pb.B @ u).max() <= 1e-13 * np.abs(pb.B @ u).max()
    gu = _host(h.apply(fvem.OP_BT, _dev(g)))
    assert np.abs(gu - pb.B.T @ g).max() <= 1e-13 * np.abs(pb.B.T @ g).max()
    y = _host(h.apply(fvem.OP_K, _dev(g)))
    assert np.abs(y - pb.K @ g).max() <= 1e-13 * np.abs(pb.K @ g).max()


@pytest.mark.parametrize("name", CASES)
def test_vcycle_fp64_matches_oracle(name, request):
    from paper_2607_17725_amd import fvem
    h, pb = hier_for(request, name)
    rng = np.random.default_rng(5)
    r = pb.null.project(rng.standard_normal(pb.K.shape[0]))
    z_ref = pb.null.project(pb.mg.vcycle(r))
    z = pb.null.project(_host(h.apply(fvem.OP_VCYCLE, _dev(r))))
    # the coarsest level solves with A_c + 1e-8 diag(A_c), whose scaled
    # condition number reaches ~1e10: rounding differences of two correct
    # summation orders grow up to ~1e-6 along near-null directions, which the
    # thin sheet's almost separated fluid layers have
    tol = 1e-6 if name.startswith("c4") else 1e-8
    assert np.linalg.norm(z - z_ref) <= tol * np.linalg.norm(z_ref)
    z32 = pb.null.project(_host(h.apply(fvem.OP_VCYCLE32, _dev(r))))
    assert np.linalg.norm(z32 - z_ref) <= 1e-4 * np.linalg.norm(z_ref)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_solve_matches_oracle(name, precision, request):
    import synth
    h, pb = hier_for(request, name)
    u = synth.normal_field(pb.vertices, 0).ravel()
    b = pb.rhs(u)
    p_ref = pb.solve_direct(u)
    p, st = h.solve(_dev(u), tol=1e-10, precision=precision, maxit=1000)
    p = _host(p)
    assert st["rel_residual"] <= 1e-10
    assert np.linalg.norm(b - pb.K @ p) <= 1e-10 * np.linalg.norm(b) * 1.01
    err = np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref)
    print(f"[gpu parity] {name} precision={precision} iters={st['iterations']} err={err:.2e}")
    assert err <= (1e-8 if precision == 0 else 1e-6)


@pytest.mark.parametrize("name", ["c2_small", "c3_small"])
def test_adjoint_matches_oracle(name, request):
    h, pb = hier_for(request, name)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(pb.K.shape[0])
    gu_ref = pb.adjoint_direct(g)
    gu, st = h.solve_adjoint(_dev(g), tol=1e-12, precision=0, maxit=1000)
    gu = _host(gu)
    assert np.linalg.norm(gu - gu_ref) <= 1e-8 * np.linalg.norm(gu_ref)


def test_autograd_function_gradient(request):
    """torch.autograd through the projection equals the oracle's exact gradient."""
    from paper_2607_17725_amd import fvem
    h, pb = hier_for(request, "c3_small")
    Fn = fvem.project_function()
    rng = np.random.default_rng(2)
    u = _dev(rng.standard_normal(3 * pb.n_vertices)).requires_grad_(True)
    w = rng.standard_normal(pb.K.shape[0])
    p = Fn.apply(u, h, 1e-12, fvem.PREC_FP64)
    loss = (p * _dev(w)).sum()
    loss.backward()
    ref = pb.adjoint_direct(w)
    assert np.linalg.norm(_host(u.grad) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_bitwise_repeatable(request):
    import synth
    h, pb = hier_for(request, "c3_small")
    u = _dev(synth.normal_field(pb.vertices, 1).ravel())
    p1, _ = h.solve(u, tol=1e-9, precision=1)
    p2, _ = h.solve(u, tol=1e-9, precision=1)
    assert torch.equal(p1, p2)


def test_error_paths(request):
    from paper_2607_17725_amd import fvem
    h, pb = hier_for(request, "c2_small")
    u = synth_u = np.random.default_rng(0).standard_normal(3 * pb.n_vertices)
    with pytest.raises(fvem.NotConverged):
        h.solve(_dev(u), tol=1e-14, maxit=1)
    # NOT_CONVERGED still writes the iterate and the stats
    p, st = h.solve(_dev(u), tol=1e-14, maxit=1, raise_not_converged=False)
    assert st["iterations"] == 1 and np.isfinite(_host(p)).all()
    bad = synth_u.copy()
    bad[3] = np.nan
    with pytest.raises(fvem.FvemError) as e:
        h.solve(_dev(bad), tol=1e-8)
    assert e.value.code == 6
    with pytest.raises(ValueError):
        h.solve(torch.zeros(5, dtype=torch.float64, device="cuda"))
    d = describe(pb)
    d["levels"][0]["cell_dof"] = d["levels"][0]["cell_dof"].copy()
    d["levels"][0]["cell_dof"][0] = pb.K.shape[0] + 5
    with pytest.raises(fvem.FvemError) as e:
        fvem.Hierarchy(d)
    assert e.value.code == 1
    # a prolongation row reaching outside its parent cell is rejected (not diffusion-free)
    d = describe(pb)
    rp, ci, va = d["levels"][0]["P"]
    ci = ci.copy()
    row0_cells = [c for c in range(len(d["levels"][0]["cell_ptr"]) - 1)
                  if 0 in d["levels"][0]["cell_dof"][d["levels"][0]["cell_ptr"][c]:d["levels"][0]["cell_ptr"][c + 1]]]
    parents = {int(d["levels"][0]["parent"][c]) for c in row0_cells}
    cp1, cd1 = d["levels"][1]["cell_ptr"], d["levels"][1]["cell_dof"]
    allowed = set()
    for E in parents:
        allowed.update(cd1[cp1[E]:cp1[E + 1]].tolist())
    outside = next(j for j in range(d["levels"][1]["n_dof"]) if j not in allowed)
    ci[rp[0]] = outside
    d["levels"][0]["P"] = (rp, ci, va)
    with pytest.raises(fvem.FvemError) as e:
        fvem.Hierarchy(d)
    assert e.value.code == 1


@pytest.mark.parametrize("name", ["c3_small", "c4_small"])
def test_whole_slice_kernel_on_every_level(name, request):
    """The oracle-sized levels normally use the row-split kernel (16 lanes per
    row); forcing the whole-slice kernel (one lane per row, the one the large
    levels run) on every level must give the same answers."""
    import synth
    from paper_2607_17725_amd import fvem
    pb = request.getfixturevalue(name)
    h = _hier(pb, small_level_rows=-1)
    rng = np.random.default_rng(5)
    r = pb.null.project(rng.standard_normal(pb.K.shape[0]))
    z_ref = pb.null.project(pb.mg.vcycle(r))
    z = pb.null.project(_host(h.apply(fvem.OP_VCYCLE, _dev(r))))
    tol = 1e-6 if name.startswith("c4") else 1e-8   # see test_vcycle_fp64_matches_oracle
    assert np.linalg.norm(z - z_ref) <= tol * np.linalg.norm(z_ref)
    z32 = pb.null.project(_host(h.apply(fvem.OP_VCYCLE32, _dev(r))))
    assert np.linalg.norm(z32 - z_ref) <= 1e-4 * np.linalg.norm(z_ref)
    u = synth.normal_field(pb.vertices, 0).ravel()
    p, st = h.solve(_dev(u), tol=1e-10, precision=1, maxit=1000)
    p_ref = pb.solve_direct(u)
    assert np.linalg.norm(_host(p) - p_ref) <= 1e-6 * np.linalg.norm(p_ref)


def test_zero_right_hand_side(request):
    """b = 0 (e.g. a divergence-free input) returns p = 0 without iterating."""
    h, pb = hier_for(request, "c3_small")
    u = torch.zeros(3 * pb.n_vertices, dtype=torch.float64, device="cuda")
    p, st = h.solve(u, tol=1e-10)
    assert st["iterations"] == 0 and st["rel_residual"] == 0.0
    assert float(p.abs().max()) == 0.0


def test_single_level_hierarchy(request):
    """A hierarchy of one level: the preconditioner is the dense solve itself."""
    import synth
    from paper_2607_17725_amd import fvem
    pb = request.getfixturevalue("c1_small")
    d = describe(pb)
    d["levels"] = d["levels"][:1]
    d["levels"][0]["parent"] = None
    d["levels"][0]["P"] = None
    h = fvem.Hierarchy(d)
    assert h.n_levels == 1
    u = synth.normal_field(pb.vertices, 0).ravel()
    p, st = h.solve(_dev(u), tol=1e-10, precision=0)
    p_ref = pb.solve_direct(u)
    assert st["iterations"] <= 3
    assert np.linalg.norm(_host(p) - p_ref) <= 1e-8 * np.linalg.norm(p_ref)


def test_obstacle_free_grid():
    """No boundary triangles: the uncut grid (every cell a plain cube), native builder."""
    import synth
    from paper_2607_17725_amd import fvem
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    V = np.zeros((0, 3))
    F = np.zeros((0, 3), dtype=np.int32)
    g = fvem.Grid(V, F, 16, 2, 5, False)
    h = fvem.Hierarchy(g)
    assert g.n_trees == 0 and g.n_dof == 33 ** 3
    u = _dev(synth.fourier_field(g.vertices, 0).ravel())
    p, st = h.solve(u, tol=1e-10, precision=1)
    assert st["rel_residual"] <= 1e-10
    # the uncut grid keeps the empty domain's mesh-independent convergence
    assert st["iterations"] <= 20
