"""Pins of oracle steps that the end-to-end identities do not reach.

* Greedy cut removal of the hierarchy (Sec. 5.2): removable cuts leave in
  increasing importance weight, and an iteration stops at the first removal
  that takes the removed weight past the budget 1/L.
* The importance weight of a cut (Sec. 5.2): the boundary-covered part of
  the cut polygon divided by the total boundary area.
* The triangle order of a background cell (Sec. 5.1): fewest crossings of a
  triangle's supporting plane with the cell's other triangles first.
* Fluid/solid classification (Sec. 5.1): the finest fluid volume equals the
  cube minus the enclosed solid volume.
* The Chebyshev bound: Gershgorin of D^-1/2 A D^-1/2.
* Dropped prolongation weights are exact zeros: an exact rational k = 2
  projector of a box with split faces has zeros exactly where the oracle
  computes rounding-level weights, and on the parity workloads every dropped
  weight sits orders of magnitude below every kept one.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.geometry import build_cell_tree, triangle_planes
from oracle.hierarchy import LevelState
from oracle.multigrid import gershgorin


# ------------------------------------------------------------------ greedy cut removal

class _Node:
    def __init__(self, nid, parent, weight=0.0, children=None):
        self.id, self.parent, self.weight, self.children = nid, parent, weight, children


class _Forest:
    def __init__(self, N, trees):
        self.N, self.trees = N, trees


def _two_trees():
    # tree A at (0,0,0): root (w 1/4) -> leaf 1, node 2 (w 1/16) -> leaves 3, 4
    A = [_Node(0, -1, 0.25, (1, 2)), _Node(1, 0), _Node(2, 0, 0.0625, (3, 4)), _Node(3, 2), _Node(4, 2)]
    # tree B at (1,0,0): root (w 1/8) -> leaves 1, 2
    B = [_Node(0, -1, 0.125, (1, 2)), _Node(1, 0), _Node(2, 0)]
    return _Forest(2, {(0, 0, 0): A, (1, 0, 0): B})


def test_remove_cuts_least_weight_first_and_strict_budget():
    # budget 0.1: A.2 (1/16, total 0.0625 <= 0.1) then B.0 (1/8, total 0.1875 > 0.1): stop
    st = LevelState(_two_trees())
    count, removed = st.remove_cuts(0.1)
    assert (count, removed) == (2, 0.1875)
    assert st.active[(0, 0, 0)] == {0} and st.active[(1, 0, 0)] == set()
    assert st.E[1, 0, 0] == 0 and st.E[0, 0, 0] == -1     # B is an uncut cube again
    # budget exactly 0.1875: the total must exceed it, so A.0 (now removable) goes too
    st = LevelState(_two_trees())
    count, removed = st.remove_cuts(0.1875)
    assert (count, removed) == (3, 0.4375)
    assert st.active[(0, 0, 0)] == set() and st.E[0, 0, 0] == 0
    # a parent becomes removable only once both children are leaves
    st = LevelState(_two_trees())
    count, _ = st.remove_cuts(0.0)
    assert count == 1 and st.active[(0, 0, 0)] == {0} and st.active[(1, 0, 0)] == {0}


def test_remove_cuts_ties_by_background_cell():
    trees = {(1, 1, 1): [_Node(0, -1, 0.5, (1, 2)), _Node(1, 0), _Node(2, 0)],
             (0, 1, 1): [_Node(0, -1, 0.5, (1, 2)), _Node(1, 0), _Node(2, 0)]}
    st = LevelState(_Forest(2, trees))
    assert st.remove_cuts(0.0) == (1, 0.5)
    assert st.active[(0, 1, 1)] == set() and st.active[(1, 1, 1)] == {0}


# ------------------------------------------------------------------ cut-cell construction

def _one_cell_tree(V, F, total_area):
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    planes = triangle_planes(V, F)
    return build_cell_tree((0, 0, 0), list(range(len(F))), V, F, planes, total_area, 1.0)


def test_importance_weight_is_boundary_covered_area():
    # a triangle in z = 0.5 whose part inside the unit cell is the square
    # [0.5, 1]^2 (area 1/4); the cut polygon itself is the whole unit square
    V = [(0.5, 0.5, 0.5), (1.5, 0.5, 0.5), (0.5, 1.5, 0.5)]
    nodes = _one_cell_tree(V, [(0, 1, 2)], total_area=2.0)
    assert nodes[0].children is not None
    assert abs(nodes[0].weight - 0.25 / 2.0) < 1e-15
    # fully inside: the whole triangle (area 0.08) counts
    V = [(0.2, 0.2, 0.5), (0.6, 0.2, 0.5), (0.2, 0.6, 0.5)]
    nodes = _one_cell_tree(V, [(0, 1, 2)], total_area=0.5)
    assert abs(nodes[0].weight - 0.08 / 0.5) < 1e-15


def test_triangle_order_fewest_plane_crossings_first():
    # A: z = 0.5 across the cell; its plane separates the vertices of B and C
    #    (2 crossings).  B: x = 0.3, y in [0.1, 0.5]; its plane crosses A only.
    #    C: y = 0.7, x in [0.5, 0.9]; its plane crosses A only.
    V = [(0.05, 0.05, 0.5), (0.95, 0.05, 0.5), (0.05, 0.95, 0.5),      # A
         (0.3, 0.1, 0.1), (0.3, 0.5, 0.1), (0.3, 0.3, 0.9),            # B
         (0.5, 0.7, 0.1), (0.9, 0.7, 0.1), (0.7, 0.7, 0.9)]            # C
    A, B, C = (0, 1, 2), (3, 4, 5), (6, 7, 8)
    for F, first in (([A, B, C], (1.0, 0.0, 0.0)), ([A, C, B], (0.0, 1.0, 0.0))):
        nodes = _one_cell_tree(V, F, total_area=1.0)
        n, _ = nodes[0].plane
        # counts A = 2, B = C = 1: the lower-indexed of B and C cuts first
        assert np.allclose(np.abs(n), first)


@pytest.mark.parametrize("fx", ["c1_small", "c3_small"])
def test_fluid_volume_and_classification(fx, request):
    from synth.shapes import signed_volume
    pb = request.getfixturevalue(fx)
    V, F = pb.boundary
    solid = abs(signed_volume(V, F))
    fluid = float(np.sum(pb.meshes[0].cell_volume))
    assert abs(fluid - (1.0 - solid)) < 1e-12
    ins = pb.forest.inside
    if fx == "c1_small":
        solid_pt = np.array([0.5, 0.5, 0.5])                 # centre of the sphere
    else:
        # centre of the upper plate: half the gap plus half the 0.05 thickness
        # along the tilted normal; the gap between the plates is fluid
        n = np.array([0.0, -np.sin(np.radians(17.0)), np.cos(np.radians(17.0))])
        solid_pt = 0.5 + (0.5 * 0.3 / pb.w.N + 0.025) * n
        assert not ins.inside(np.array([0.5, 0.5, 0.5]))
    assert ins.inside(solid_pt)
    assert not ins.inside(np.array([0.03, 0.04, 0.05]))


# ------------------------------------------------------------------ smoother bound

def test_gershgorin_bound_of_scaled_matrix():
    A = sp.csr_matrix(np.array([[4.0, -2.0, 0.0], [-2.0, 1.0, 0.5], [0.0, 0.5, 9.0]]))
    dinv = 1.0 / A.diagonal()
    # D^-1/2 A D^-1/2 = [[1, -1, 0], [-1, 1, 1/6], [0, 1/6, 1]]: row sums 2, 13/6, 7/6
    assert abs(gershgorin(A, dinv) - 13.0 / 6.0) < 1e-15
    assert abs(gershgorin(A) - 9.5) < 1e-15


# ------------------------------------------------------------------ dropped prolongation weights

def _split_box_faces():
    """Cell [0,2]^3 whose face x = 0 is split into 4 squares (hanging vertices
    on the faces y = 0, 2 and z = 0, 2), as in a coarse cube beside finer cells."""
    F = []
    for y0, z0 in ((0, 0), (1, 0), (0, 1), (1, 1)):
        F.append([(0, y0, z0), (0, y0, z0 + 1), (0, y0 + 1, z0 + 1), (0, y0 + 1, z0)])
    F.append([(2, 0, 0), (2, 2, 0), (2, 2, 2), (2, 0, 2)])
    F.append([(0, 0, 0), (2, 0, 0), (2, 0, 2), (0, 0, 2), (0, 0, 1)])
    F.append([(0, 2, 0), (0, 2, 1), (0, 2, 2), (2, 2, 2), (2, 2, 0)])
    F.append([(0, 0, 0), (0, 1, 0), (0, 2, 0), (2, 2, 0), (2, 0, 0)])
    F.append([(0, 0, 2), (2, 0, 2), (2, 2, 2), (0, 2, 2), (0, 1, 2)])
    return F


def test_cell_projector_exact_and_zero_weights_exact():
    """The oracle's k = 2 cell projection equals an exact rational evaluation,
    and its rounding-level weights are exactly the exact zeros."""
    from exact_vem import ExactBoxCell
    from oracle.quadrature import polyhedron_rule
    from oracle.vem import StandaloneCell, cell_projector
    from oracle.geometry import make_box
    F = _split_box_faces()
    ex = ExactBoxCell(F, (0, 0, 0), (2, 2, 2))
    Pe, mono = ex.projector()
    g = StandaloneCell([np.array(f, dtype=np.float64) for f in F])
    assert [tuple(g.X[v]) for v in g.verts] == [tuple(float(c) for c in p) for p in ex.verts]
    Pis, _, _ = cell_projector(g, 2)
    rows = []
    for p in ((1, 1, 1), (1, 1, 0.5), (0.5, 1, 1), (1, 0.5, 1), (0.5, 0.5, 0.5), (1.5, 1, 1)):
        rows.append((ex.value_weights(Pe, mono, p), g.basis.mono(np.array(p, dtype=np.float64), 2)[0] @ Pis))
    for lo in ((0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)):
        hi = tuple(c + 1 for c in lo)
        qp, qw = polyhedron_rule([f[0] for f in make_box(np.array(lo, float), np.array(hi, float))])
        rows.append((ex.mean_weights(Pe, mono, lo, hi), (qw @ g.basis.mono(qp, 2) / qw.sum()) @ Pis))
    zeros = 0
    for we, wo in rows:
        we = np.array([float(v) for v in we])
        scale = np.abs(we).max()
        assert np.abs(we - wo).max() <= 1e-13 * scale
        exact_zero = we == 0.0
        dropped = np.abs(wo) <= 1e-13 * np.abs(wo).max()      # the oracle's rule
        assert np.array_equal(exact_zero, dropped)
        zeros += int(exact_zero.sum())
    assert zeros > 100


@pytest.mark.parametrize("fx", ["c1_small", "c3_small"])
def test_dropped_weights_are_separated_from_kept(fx, request):
    """Every weight the rule drops is at rounding level, far below every kept
    weight; every removed coarse column is rounding residue."""
    pb = request.getfixturevalue(fx)
    for P_raw, used in pb.P_raw:
        P = P_raw.tocsr()
        rowmax = np.asarray(abs(P).max(axis=1).todense()).ravel()
        coo = P.tocoo()
        rel = np.abs(coo.data) / rowmax[coo.row]
        dropped = rel <= 1e-13
        assert not np.any((rel > 1e-13) & (rel <= 1e-9))
        assert np.abs(coo.data[dropped]).max(initial=0.0) <= 1e-14
        colmax = np.asarray(abs(P).max(axis=0).todense()).ravel()
        assert colmax[~used].max(initial=0.0) <= 1e-14
        assert colmax[used].min() >= 1e-9


def test_dropped_weights_below_sheet_rounding(c4_small):
    """On the 1e-5-thin sheet the local projections of sliver cells carry
    rounding up to ~1e-9 of a row's largest weight, so weights there form a
    continuum down from that level; the rule drops only what lies four orders
    below it, which changes no reproduced polynomial value beyond 1e-12, and
    the removed columns stay two orders below every kept one."""
    from test_oracle_global import _dof_values, _poly
    pb = c4_small
    q, _ = _poly(2, 5)
    for t, (P_raw, used) in enumerate(pb.P_raw):
        P = P_raw.tocsr()
        rowmax = np.asarray(abs(P).max(axis=1).todense()).ravel()
        colmax = np.asarray(abs(P).max(axis=0).todense()).ravel()
        assert colmax[~used].max(initial=0.0) <= 1e-12
        assert colmax[used].min() >= 1e-10
        Dc = _dof_values(pb, t + 1, q)
        Dfull = np.zeros(P.shape[1])
        Dfull[np.nonzero(used)[0]] = Dc
        diff = P @ Dfull - pb.P[t] @ Dc
        assert np.abs(diff).max() <= 1e-12 * np.abs(Dc).max()
        coo = P.tocoo()
        kept = np.abs(coo.data) > 1e-13 * rowmax[coo.row]
        assert pb.P[t].nnz == int(kept[used[coo.col]].sum())


# ------------------------------------------------------------------ naive prolongation (ablation)

def test_naive_prolongation_reproduces_and_diffuses():
    """The naive prolongation of Sec. 4 reproduces quadratics like the
    diffusion-free one, but its Galerkin operators couple DOFs of different
    coarse cells and grow denser level by level (the paper's diffusion)."""
    from conftest import oracle_problem
    from test_oracle_global import _dof_values, _poly
    pn = oracle_problem("c3", 8, naive_prolongation=True)
    pd = oracle_problem("c3", 8)
    q, _ = _poly(2, 5)
    for t, P in enumerate(pn.P):
        Dc, Df = _dof_values(pn, t + 1, q), _dof_values(pn, t, q)
        assert np.abs(P @ Dc - Df).max() < 1e-11 * max(np.abs(Df).max(), 1.0)
    An, Ad = pn.mg.A, pd.mg.A
    assert An[0].nnz == Ad[0].nnz
    for l in range(1, len(An)):
        assert An[l].nnz > 2 * Ad[l].nnz
    # coupling outside the coarse cliques on the first coarse level
    d = pn.dofs[1]
    allowed = set()
    for c in range(len(pn.meshes[1].cell_faces)):
        ids = d.free[d.cell_dofs(c)]
        ids = ids[ids >= 0]
        allowed.update((int(i), int(j)) for i in ids for j in ids)
    coo = An[1].tocoo()
    big = np.abs(coo.data) > 1e-12 * np.abs(coo.data).max()
    outside = sum((int(i), int(j)) not in allowed for i, j in zip(coo.row[big], coo.col[big]))
    assert outside > 0.5 * big.sum()
