"""The naive prolongation (the Sec. 4 ablation) through the library.

The oracle's naive P (rows reaching DOFs of neighbouring coarse cells) goes
to the library with the general Galerkin option, which forms P^T A P by
sparse products on the host; the element-wise path must refuse it.  The
coarse operators, one FP64 V-cycle and the solve are compared with the
oracle's, with the tolerances of the diffusion-free parity tests.
"""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle_desc import describe

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.fixture(scope="module")
def naive():
    from paper_2607_17725_amd import fvem
    pb = oracle_problem("c3", 8, naive_prolongation=True)
    print("[gpu naive] building the naive-prolongation hierarchy", flush=True)
    h = fvem.Hierarchy(describe(pb), galerkin_general=True, lattice_min_fraction=1e-6)
    return h, pb


def test_elementwise_path_refuses_naive_P():
    from paper_2607_17725_amd import fvem
    pb = oracle_problem("c3", 8, naive_prolongation=True)
    with pytest.raises(fvem.FvemError, match="not diffusion-free"):
        fvem.Hierarchy(describe(pb))


def test_naive_operators_vcycle_and_solve(naive):
    import scipy.sparse as sp
    import synth
    from paper_2607_17725_amd import fvem
    h, pb = naive
    mg = pb.mg
    for l in range(1, h.n_levels):
        rp, ci, va = h.level_matrix(l)
        A = sp.csr_matrix((va, ci, rp), shape=mg.A[l].shape)
        assert abs(A - mg.A[l]).max() <= 1e-12 * abs(mg.A[l]).max()
        print(f"[gpu naive] level {l}: nnz {A.nnz}", flush=True)
    r = pb.null.project(np.random.default_rng(9).standard_normal(h.n_dof))
    z = h.apply(fvem.OP_VCYCLE, _dev(r)).cpu().numpy()
    zr = pb.null.project(mg.vcycle(r))
    assert np.linalg.norm(pb.null.project(z) - zr) <= 1e-8 * np.linalg.norm(zr)
    u = synth.fourier_field(pb.vertices, 0).ravel()
    ref = pb.solve_direct(u)
    for prec in (fvem.PREC_FP64, fvem.PREC_MIXED):
        p, st = h.solve(_dev(u), tol=1e-10, precision=prec)
        p = p.cpu().numpy()
        b = pb.rhs(u)
        assert np.linalg.norm(b - pb.K @ p) <= 1.01e-10 * np.linalg.norm(b)
        assert np.linalg.norm(p - ref) <= 1e-6 * np.linalg.norm(ref)
        print(f"[gpu naive] precision {prec}: {st['iterations']} iterations", flush=True)
