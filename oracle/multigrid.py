"""Galerkin geometric multigrid and preconditioned CG in FP64 (Sec. 4 and Sec. 6).

* Coarse operators: A_{l+1} = R_l A_l P_l with R_l = P_l^T (Galerkin, the
  paper's coarse-operator definition).
* Smoother: Chebyshev semi-iteration (Saad, Iterative Methods for Sparse
  Linear Systems, Alg. 12.1) of degree 5 on D^-1 A (D = diag A) over
  [lmax/30, lmax], lmax the Gershgorin bound of the similar matrix
  D^-1/2 A D^-1/2, max_i sum_j |a_ij| / sqrt(a_ii a_jj), which stays below
  the row length even where a coarse diagonal is tiny.  The
  paper specifies "the Chebyshev smoother with default parameters" of a
  library that is not available; this is the reading taken (parity unpinned
  against that library).  The diagonal scaling is needed on cut-cell grids
  with 1e-5-thin cells, whose diagonal entries exceed the regular cells' by
  ~1e6: an unscaled polynomial over [lmax/30, lmax] leaves the regular
  cells' error untouched and the outer CG stalls.
* Cycle: V(1,1), zero initial guess on every level (reading; the paper gives
  no cycle details).
* Coarsest level: dense Cholesky of A_c + 1e-8 diag(A_c) (reading; the
  paper is silent on the coarse solver).  A_c is only positive
  semi-definite: besides the constants of pure-Neumann components, coarse
  cells reaching into the solid carry DOFs that act on the fine grid only
  through the cell projection, so some combinations v have P v = 0.  Every
  restricted right-hand side is orthogonal to those null vectors (by
  induction from the zero-mean fine residual: v.P^T r = (P v).r = 0), the
  shifted matrix is positive definite, and the components the shift creates
  along null(P) vanish after prolongation; genuine modes (>= 1e-7 of the
  largest eigenvalue in the workloads here) change by under 10%.
* Outer solve: CG preconditioned by one V-cycle, with the Polak-Ribiere
  beta (flexible form), x0 = 0, true-residual replacement every 10
  iterations, stopping on ||b - K x|| / ||b|| <= tol.  On pure-Neumann
  components b, the preconditioned residual and the result are kept at
  zero DOF mean.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def galerkin(A, P):
    R = P.T.tocsr()
    Ac = (R @ A @ P).tocsr()
    Ac.sum_duplicates()
    Ac.sort_indices()
    return Ac


def gershgorin(A, dinv=None):
    """Gershgorin bound of A, or with ``dinv`` of D^-1/2 A D^-1/2 (the spectrum of D^-1 A)."""
    if dinv is None:
        return float(np.asarray(np.abs(A).sum(axis=1)).ravel().max())
    s = np.sqrt(np.abs(dinv))
    S = sp.diags(s) @ abs(A) @ sp.diags(s)
    return float(np.asarray(S.sum(axis=1)).ravel().max())


class NullSpace:
    """Indicator vectors of the floating (zero row-sum) components of a matrix graph."""

    def __init__(self, A, rtol=1e-9):
        n = A.shape[0]
        ncomp, lab = connected_components(A, directed=False)
        rs = np.abs(A @ np.ones(n))
        scale = np.abs(A).sum(axis=1).A1 if sp.issparse(A) else np.abs(A).sum(axis=1)
        self.labels = lab
        self.floating = []
        for c in range(ncomp):
            idx = np.nonzero(lab == c)[0]
            if rs[idx].max() <= rtol * scale[idx].max():
                self.floating.append(idx)

    def project(self, v):
        v = v.copy()
        for idx in self.floating:
            v[idx] -= v[idx].mean()
        return v


def chebyshev(A, b, x, lmax, degree=5, lower=1.0 / 30.0, x_is_zero=False, dinv=None):
    """Degree-``degree`` Chebyshev smoothing of A x = b preconditioned by diag(dinv)."""
    if dinv is None:
        dinv = np.ones(A.shape[0])
    lo, hi = lower * lmax, lmax
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b.copy() if x_is_zero else b - A @ x
    d = dinv * r / theta
    x = d.copy() if x_is_zero else x + d
    for _ in range(degree - 1):
        r = b - A @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        x = x + d
        rho = rho_new
    return x


COARSE_SHIFT = 1e-8


class CoarseSolver:
    def __init__(self, A, shift=COARSE_SHIFT):
        Ad = A.toarray() if sp.issparse(A) else np.array(A)
        self.n = len(Ad)
        M = Ad + shift * np.diag(np.diag(Ad))
        self.L = np.linalg.cholesky(M)

    def solve(self, b):
        from scipy.linalg import solve_triangular
        y = solve_triangular(self.L, b, lower=True)
        return solve_triangular(self.L.T, y, lower=False)


class Hierarchy:
    def __init__(self, A0, Ps, degree=5, lower=1.0 / 30.0):
        self.A = [A0.tocsr()]
        self.P = list(Ps)
        for P in self.P:
            self.A.append(galerkin(self.A[-1], P))
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        self.lmax = [gershgorin(A, di) for A, di in zip(self.A, self.dinv)]
        self.degree, self.lower = degree, lower
        self.coarse = CoarseSolver(self.A[-1])

    def vcycle(self, b, level=0):
        A = self.A[level]
        if level == len(self.A) - 1:
            return self.coarse.solve(b)
        di = self.dinv[level]
        x = chebyshev(A, b, None, self.lmax[level], self.degree, self.lower, x_is_zero=True, dinv=di)
        r = b - A @ x
        bc = self.P[level].T @ r
        xc = self.vcycle(bc, level + 1)
        x = x + self.P[level] @ xc
        return chebyshev(A, b, x, self.lmax[level], self.degree, self.lower, dinv=di)


def pcg(K, b, precond, null=None, tol=1e-10, maxit=500, replace_every=10):
    """Flexible PCG; returns (x, iterations, true relative residual history)."""
    proj = (lambda v: null.project(v)) if null is not None else (lambda v: v)
    b = proj(b)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0:
        return x, 0, [0.0]
    r = b.copy()
    z = proj(precond(r))
    p = z.copy()
    rz = r @ z
    hist = [1.0]
    it = 0
    while it < maxit:
        q = K @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if it % replace_every == 0:
            r = b - K @ x
        rel = np.linalg.norm(r) / nb
        if rel <= tol:
            r = b - K @ x
            rel = np.linalg.norm(r) / nb
            hist.append(rel)
            if rel <= tol:
                break
        else:
            hist.append(rel)
        z_new = proj(precond(r))
        beta = (r @ (z_new - z)) / rz
        rz = r @ z_new
        z = z_new
        p = z + beta * p
    return proj(x), it, hist


def direct_solve(K, b, null=None):
    """Exact reference: sparse LU with one DOF pinned per floating component."""
    from scipy.sparse.linalg import splu
    n = K.shape[0]
    b = null.project(b) if null is not None else b.copy()
    pins = [idx[0] for idx in (null.floating if null is not None else [])]
    if pins:
        keep = np.setdiff1d(np.arange(n), pins)
        Kr = K[keep][:, keep].tocsc()
        x = np.zeros(n)
        x[keep] = splu(Kr).solve(b[keep])
        return null.project(x)
    return splu(K.tocsc()).solve(b)
