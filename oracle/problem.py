"""End-to-end oracle problem: grid, hierarchy, operators and reference solves.

The reference answer of the pressure projection (Sec. 3.1, K p = r) for a
velocity u is p* = K^+ P_perp B u: the unique solution with zero DOF mean on
every pure-Neumann component, or of the Dirichlet-reduced system when the
top face carries p = 0.  The MG-PCG only reaches p* faster, to a tolerance.
"""
import numpy as np

from .assemble import Assembly, Dofs
from .hierarchy import build_hierarchy
from .multigrid import Hierarchy, NullSpace, direct_solve, pcg
from .prolong import build_prolongation


UNUSED_TOL = 1e-10


def _dof_count(k):
    def f(mesh):
        if k == 1:
            return len(mesh.X)
        return len(mesh.X) + len(mesh.edges) + len(mesh.faces) + len(mesh.cell_faces)
    return f


class Problem:
    def __init__(self, workload, coarse_max=16384, max_levels=12, with_velocity=True, naive_prolongation=False):
        w = workload
        self.w = w
        self.k = w.k
        V, F = w.mesh()
        self.boundary = (V, F)
        self.forest, levels, self.parents = build_hierarchy(
            V, F, w.N, w.levels, coarse_max=coarse_max, dof_count=_dof_count(w.k), max_levels=max_levels)
        self.meshes = [lv[2] for lv in levels]
        self.dofs = [Dofs(m, w.k, w.dirichlet_top) for m in self.meshes]
        self.asm = Assembly(self.meshes[0], self.dofs[0], with_velocity)
        self.K = self.asm.K
        self.B = self.asm.B if with_velocity else None
        self.P = []
        self.P_raw = []
        self.host_kind = []
        for t in range(len(self.meshes) - 1):
            P, hk, P_raw = build_prolongation(self.meshes[t], self.dofs[t], self.meshes[t + 1],
                                              self.dofs[t + 1], self.parents[t], return_raw=True,
                                              naive=naive_prolongation)
            # Reading of this build (not a statement of the paper): a coarse
            # DOF whose prolongation column is zero carries no information
            # and is removed.  Sec. 5.2 argues that nestedness keeps the
            # restriction full-rank, but coarse cells here keep their solid
            # part (the coarse-inclusion reading), and some coarse DOFs then
            # have every weight equal to zero in exact arithmetic (e.g. the
            # DOFs of sub-faces of a split coarse face away from all fine
            # fluid cells).  Their computed weights are rounding residue,
            # at most ~1e-15 here; a largest weight <= 1e-10 marks them.
            used = np.asarray(np.abs(P).max(axis=0).todense()).ravel() > UNUSED_TOL
            self.P_raw.append((P_raw, used))
            if not used.all():
                self.dofs[t + 1].deactivate(self.dofs[t + 1].free_ids[~used])
                P = P[:, np.nonzero(used)[0]].tocsr()
            self.P.append(P)
            self.host_kind.append(hk)
        self.null = NullSpace(self.K)
        self._mg = None

    @property
    def mg(self):
        if self._mg is None:
            self._mg = Hierarchy(self.K, self.P)
        return self._mg

    @property
    def n_vertices(self):
        return self.dofs[0].nv

    @property
    def vertices(self):
        return self.meshes[0].X

    def rhs(self, u):
        return self.null.project(self.B @ np.asarray(u, dtype=np.float64).ravel())

    def solve_direct(self, u=None, b=None):
        if b is None:
            b = self.rhs(u)
        return direct_solve(self.K, b, self.null)

    def solve_mgpcg(self, u=None, b=None, tol=1e-10, maxit=500):
        if b is None:
            b = self.rhs(u)
        return pcg(self.K, b, self.mg.vcycle, self.null, tol=tol, maxit=maxit)

    def adjoint_direct(self, gp):
        """g_u = B^T P_perp K^+ P_perp g_p (the transpose of u -> p*)."""
        lam = direct_solve(self.K, self.null.project(np.asarray(gp, dtype=np.float64)), self.null)
        return self.B.T @ self.null.project(lam)

    def full_pressure(self, p_free, level=0):
        d = self.dofs[level]
        out = np.zeros(d.n)
        out[d.free_ids] = p_free
        return out
