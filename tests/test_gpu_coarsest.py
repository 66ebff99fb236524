"""The coarsest-level dense solve against a LAPACK solve of the same operator.

With one level the whole level-0 operator is the coarsest one and the
preconditioner is z = G r, where G = (A + 1e-8 diag A)^+ comes from the
blocked Cholesky, the triangular inverse and G = X^T X, all on the GPU (the
trailing updates and the product on FP64 MFMA).  The operator is read back
column by column through K applications and numpy solves the same shifted
system:
- the sphere at 8^3 with its Dirichlet top (k = 1, 1,366 DOFs: positive
  definite; 21 full 64-blocks and a ragged one);
- the plates at 8^3, k = 2 (6,959 DOFs, pure Neumann: positive
  semi-definite), on a right-hand side with zero mean on every fluid
  component; both results are compared after the same projection.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,N,tol", [("c1", 8, 1e-10), ("c3", 8, 1e-7)])
def test_coarsest_solve_matches_lapack(name, N, tol):
    import synth
    from paper_2607_17725_amd import fvem
    w = synth.get_config(name, N=N)
    V, F = w.mesh()
    print(f"[gpu coarsest] {name}@{N}: one-level hierarchy", flush=True)
    g = fvem.Grid(V, F, w.N, w.k, 1, w.dirichlet_top)
    h = fvem.Hierarchy(g)
    n = h.n_dof
    K = np.empty((n, n))
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    for j in range(n):
        e.zero_()
        e[j] = 1.0
        K[:, j] = h.apply(fvem.OP_K, e).cpu().numpy()
    assert np.allclose(K, K.T, rtol=0, atol=1e-12 * np.abs(K).max())
    free = np.diag(K) != 0.0          # level-order holes have empty rows
    rng = np.random.default_rng(3)
    r = torch.as_tensor(rng.standard_normal(n), device="cuda")
    r[torch.as_tensor(~free, device="cuda")] = 0.0
    r = h.apply(fvem.OP_PROJECT, r)
    z = h.apply(fvem.OP_VCYCLE, r).cpu().numpy()
    Kf = K[np.ix_(free, free)]
    Ks = Kf + 1e-8 * np.diag(np.diag(Kf))
    zf = np.zeros(n)
    zf[free] = np.linalg.solve(Ks, r.cpu().numpy()[free])
    zref = h.apply(fvem.OP_PROJECT, torch.as_tensor(zf, device="cuda")).cpu().numpy()
    zgot = h.apply(fvem.OP_PROJECT, torch.as_tensor(z, device="cuda")).cpu().numpy()
    err = np.linalg.norm(zgot - zref) / np.linalg.norm(zref)
    print(f"[gpu coarsest] {name}@{N}: n = {n}, |z - z_lapack| / |z_lapack| = {err:.2e}", flush=True)
    assert np.all(z[~free] == 0.0)
    assert err <= tol
