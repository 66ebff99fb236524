"""Cut-cell forest and the nested, boundary-aware grid hierarchy (Sec. 5.1-5.2).

Level 0 is the finest grid.  One coarsening iteration (level t -> t+1):
1. aggregate every aligned 2x2x2 block of equal uncut cubes into one cube
   ("standard geometric multigrid practice"),
2. greedily remove removable cuts (both children are current leaves) in
   increasing importance weight until the removed weight of this iteration
   exceeds 1/L,
3. keep the current cells that contain at least one finest fluid cell (the
   coarse cell keeps its whole convex region, solid part included).

Readings taken where the paper is silent (conventions, parity unpinned):
* aggregation keeps the grid 2:1 balanced: a block is merged only when every
  cell touching it (face, edge or corner) is at least as large as the block's
  members, which bounds the number of faces a coarse cube can have; cells of a
  background cell that still holds cuts count as size 1;
* the removal budget 1/L is per iteration; ties broken by (weight, background
  cell index, node id);
* coarsening continues past L-1 iterations while the coarsest level has more
  than ``coarse_max`` DOFs (and something can still be coarsened).
"""
import heapq
import numpy as np

from .geometry import (associate_triangles, build_cell_tree, triangle_planes,
                       InsideTest, make_box)
from .mesh import Tile, conform


class Forest:
    """Binary space partition trees of every cut background cell."""

    def __init__(self, V, F, N):
        self.N = N
        self.h = 1.0 / N
        planes = triangle_planes(V, F)
        self.total_area = float(planes[2].sum())
        assoc = associate_triangles(V, F, N)
        self.inside = InsideTest(V, F, N)
        self.trees = {}
        for bg in sorted(assoc):
            nodes = build_cell_tree(bg, assoc[bg], V, F, planes, self.total_area, self.h)
            if len(nodes) > 1:
                self.trees[bg] = nodes
        # classify leaves and uncut cells
        self.bg_fluid = np.zeros((N, N, N), dtype=bool)
        for bg, nodes in self.trees.items():
            for nd in nodes:
                if nd.children is None:
                    nd.fluid = not self.inside.inside(nd.centroid)
            self._propagate_fluid(nodes)
            self.bg_fluid[bg] = nodes[0].fluid
        cols = self.inside.cols
        for i in range(N):
            for j in range(N):
                if (i, j) not in cols:
                    for k in range(N):
                        if (i, j, k) not in self.trees:
                            self.bg_fluid[i, j, k] = True
                    continue
                for k in range(N):
                    if (i, j, k) in self.trees:
                        continue
                    p = (np.array([i, j, k]) + 0.5) * self.h
                    self.bg_fluid[i, j, k] = not self.inside.inside(p)

    @staticmethod
    def _propagate_fluid(nodes):
        for nd in reversed(nodes):
            if nd.children is not None:
                nd.fluid = nodes[nd.children[0]].fluid or nodes[nd.children[1]].fluid


class LevelState:
    """Current cells: active cuts per tree, cube exponents per background cell."""

    def __init__(self, forest):
        N = forest.N
        self.forest = forest
        self.active = {bg: {nd.id for nd in nodes if nd.children is not None}
                       for bg, nodes in forest.trees.items()}
        self.E = np.zeros((N, N, N), dtype=np.int64)
        for bg in forest.trees:
            self.E[bg] = -1

    def copy(self):
        s = LevelState.__new__(LevelState)
        s.forest = self.forest
        s.active = {bg: set(a) for bg, a in self.active.items()}
        s.E = self.E.copy()
        return s

    def leaves(self, bg):
        """Current leaves of the tree of ``bg`` (node ids)."""
        nodes = self.forest.trees[bg]
        act = self.active[bg]
        out = []
        stack = [0]
        while stack:
            i = stack.pop()
            if i in act:
                stack += list(nodes[i].children[::-1])
            else:
                out.append(i)
        return sorted(out)

    def tiles(self):
        """The convex tiling of the unit cube at this level, plus lookup maps."""
        f = self.forest
        N, h = f.N, f.h
        tiles = []
        leaf_tile = {}
        cube_tile = {}
        for bg in sorted(self.active):
            if self.E[bg] >= 0:
                continue
            nodes = f.trees[bg]
            for nid in self.leaves(bg):
                nd = nodes[nid]
                leaf_tile[(bg, nid)] = len(tiles)
                tiles.append(Tile(nd.faces, bool(nd.fluid), bg, tuple(b + 1 for b in bg), 0, ("n", bg, nid)))
        seen = np.zeros((N, N, N), dtype=bool)
        for i in range(N):
            for j in range(N):
                for k in range(N):
                    s = self.E[i, j, k]
                    if s < 0 or seen[i, j, k]:
                        continue
                    w = 1 << s
                    lo = (i - i % w, j - j % w, k - k % w)
                    hi = (lo[0] + w, lo[1] + w, lo[2] + w)
                    seen[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
                    fluid = bool(f.bg_fluid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].any())
                    cube_tile[lo] = len(tiles)
                    tiles.append(Tile(make_box(np.array(lo) * h, np.array(hi) * h), fluid, lo, hi, w,
                                      ("c", s, lo)))
        return tiles, leaf_tile, cube_tile

    def aggregate(self):
        """One pass of balanced 2x2x2 aggregation of equal uncut cubes."""
        N = self.forest.N
        E = self.E
        eff = np.where(E < 0, 0, E)
        merges = []
        smax = int(E.max())
        for s in range(0, smax + 1):
            w = 1 << (s + 1)
            if w > N:
                break
            for i in range(0, N, w):
                for j in range(0, N, w):
                    for k in range(0, N, w):
                        blk = E[i:i + w, j:j + w, k:k + w]
                        if not np.all(blk == s):
                            continue
                        ex = eff[max(i - 1, 0):i + w + 1, max(j - 1, 0):j + w + 1, max(k - 1, 0):k + w + 1]
                        if ex.min() >= s:
                            merges.append((s, i, j, k))
        for s, i, j, k in merges:
            w = 1 << (s + 1)
            self.E[i:i + w, j:j + w, k:k + w] = s + 1
        return len(merges)

    def remove_cuts(self, budget):
        """Greedy removal of removable cuts of least weight until removed > budget."""
        f = self.forest
        N = f.N
        heap = []

        def removable(bg, nid):
            nd = f.trees[bg][nid]
            act = self.active[bg]
            return nid in act and nd.children[0] not in act and nd.children[1] not in act

        for bg, act in self.active.items():
            for nid in act:
                if removable(bg, nid):
                    lin = (bg[0] * N + bg[1]) * N + bg[2]
                    heapq.heappush(heap, (f.trees[bg][nid].weight, lin, nid, bg))
        removed = 0.0
        count = 0
        while heap and removed <= budget:
            w, lin, nid, bg = heapq.heappop(heap)
            self.active[bg].discard(nid)
            removed += w
            count += 1
            par = f.trees[bg][nid].parent
            if par >= 0 and removable(bg, par):
                heapq.heappush(heap, (f.trees[bg][par].weight, lin, par, bg))
            if not self.active[bg]:
                self.E[bg] = 0
        return count, removed


def coarse_parent(state_f, state_c, tile_f, leaf_tile_c, cube_tile_c):
    """Index of the coarse tile containing fine tile ``tile_f``."""
    key = tile_f.key
    f = state_c.forest
    if key[0] == "n":
        _, bg, nid = key
        if state_c.E[bg] < 0:
            act = state_c.active[bg]
            nodes = f.trees[bg]
            # ancestor-or-self that is a current leaf
            path = []
            x = nid
            while x >= 0:
                path.append(x)
                x = nodes[x].parent
            for x in reversed(path):
                if x not in act:
                    return leaf_tile_c[(bg, x)]
            raise RuntimeError("no current leaf above node")
        corner = bg
    else:
        corner = key[2]
    s = state_c.E[corner]
    w = 1 << s
    lo = tuple(c - c % w for c in corner)
    return cube_tile_c[lo]


def build_hierarchy(V, F, N, L, coarse_max=16384, k=1, dof_count=None, max_levels=12):
    """Return (forest, [(state, tiles, mesh, leaf_tile, cube_tile)], parents).

    ``parents[t]`` maps each fluid cell of level t to its coarse cell at t+1.
    ``dof_count(mesh)`` gives the DOF count used for the continue-coarsening test.
    """
    forest = Forest(V, F, N)
    state = LevelState(forest)
    levels = []
    tiles, lt, ct = state.tiles()
    mesh = conform(tiles, N)
    levels.append((state, tiles, mesh, lt, ct))
    parents = []
    t = 0
    while True:
        n_here = dof_count(levels[-1][2]) if dof_count else len(levels[-1][2].cell_faces)
        if t >= L - 1 and n_here <= coarse_max:
            break
        if len(levels) >= max_levels:
            break
        nstate = state.copy()
        nagg = nstate.aggregate()
        nrem, _ = nstate.remove_cuts(1.0 / L)
        if nagg == 0 and nrem == 0:
            break
        ntiles, nlt, nct = nstate.tiles()
        nmesh = conform(ntiles, N)
        fine_tiles = levels[-1][1]
        fine_mesh = levels[-1][2]
        coarse_cell_of_tile = {ti: ci for ci, ti in enumerate(nmesh.cell_tiles)}
        par = np.array([coarse_cell_of_tile[coarse_parent(state, nstate, fine_tiles[ti], nlt, nct)]
                        for ti in fine_mesh.cell_tiles], dtype=np.int64)
        parents.append(par)
        levels.append((nstate, ntiles, nmesh, nlt, nct))
        state = nstate
        t += 1
    return forest, levels, parents
