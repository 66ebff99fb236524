// Native grid builder: binary-space cut cells, nested boundary-aware
// hierarchy, conforming VEM meshes, element operators and the
// diffusion-free prolongation (paper Sec. 3-5), producing the problem
// description consumed by fvem_hierarchy_build.
//
// Readings where the paper is silent (shared conventions, stated once):
//  * triangle/cell association by exact triangle-box overlap; triangles of
//    a cell ordered by how many other triangles of the cell their plane
//    crosses, ties by index; cuts leaving a part below 1e-12 volume skipped;
//    a triangle follows a cut into each part where its clipped area exceeds
//    1e-14 h^2; triangles coplanar with a cut are consumed by it;
//  * leaves classified by the winding number of the boundary mesh at their
//    centroid (ray cast);
//  * coarsening: aligned 2x2x2 blocks of equal uncut cubes merge when every
//    cell touching the block is at least as large (2:1 balance), then the
//    least-weight removable cuts are removed until the removed weight of the
//    iteration exceeds 1/L; coarse cells keep their whole convex region;
//    coarsening continues past L-1 iterations while the coarsest level has
//    more DOFs than the dense coarse-solver limit;
//  * conforming faces are the overlaps of coplanar opposite facets of
//    neighbouring cells of the full (fluid + solid) tiling, with T-junction
//    vertices inserted; coarse DOFs the prolongation never uses are dropped.
#include <parallel/algorithm>
#include "grid.hpp"
#include "progress.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <omp.h>
#include <functional>
#include <queue>
#include <stdexcept>
#include <unordered_map>

namespace fvem::grid {

using geo::cross;
using geo::dot;
using geo::norm;
using geo::Polyhedron;
using geo::V3;

namespace {

constexpr double kMinVolume = 1e-12;
constexpr double kPlaneTol = 1e-12;
// vertices closer than this are one vertex: the same intersection reached
// through different clipping sequences can differ by ~1e-12 where nearly
// parallel planes meet; distinct vertices of the scenes stay above 1e-9
constexpr double kVertTol = 1e-10;

// Open-addressing map from 64-bit keys to int32 values, for the
// sequential numbering passes (no per-entry allocation).  EMPTY is never a
// key: callers map it elsewhere.
struct FlatMap {
  static constexpr uint64_t EMPTY = ~0ULL;
  std::vector<uint64_t> key;
  std::vector<int32_t> val;
  uint64_t mask = 0;
  size_t n = 0;
  explicit FlatMap(size_t expect) {
    size_t cap = 16;
    while (cap < 2 * expect) cap <<= 1;
    key.assign(cap, EMPTY);
    val.assign(cap, -1);
    mask = cap - 1;
  }
  static uint64_t spread(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    return x ^ (x >> 33);
  }
  // the value slot of k, inserted (value -1) when absent
  int32_t *find_or_insert(uint64_t k, bool *inserted) {
    if (2 * (n + 1) > key.size()) grow();
    uint64_t i = spread(k) & mask;
    while (key[i] != EMPTY) {
      if (key[i] == k) {
        *inserted = false;
        return &val[i];
      }
      i = (i + 1) & mask;
    }
    key[i] = k;
    ++n;
    *inserted = true;
    return &val[i];
  }
  void grow() {
    std::vector<uint64_t> k2;
    std::vector<int32_t> v2;
    k2.swap(key);
    v2.swap(val);
    key.assign(2 * k2.size(), EMPTY);
    val.assign(2 * k2.size(), -1);
    mask = key.size() - 1;
    for (size_t j = 0; j < k2.size(); ++j) {
      if (k2[j] == EMPTY) continue;
      uint64_t i = spread(k2[j]) & mask;
      while (key[i] != EMPTY) i = (i + 1) & mask;
      key[i] = k2[j];
      val[i] = v2[j];
    }
  }
};

struct Node {
  Polyhedron poly;
  V3 n;
  double d = 0;
  int child[2] = {-1, -1};
  int parent = -1;
  double w = 0;
  bool fluid = false;
  double vol = 0;
  V3 cen;
};

struct Tree {
  int64_t bg = 0;
  std::vector<Node> nodes;
};

struct Tile {
  int type = 0;   // 0 tree leaf, 1 cube
  int32_t tree = -1, node = -1;
  int s = 0;      // cube exponent
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bool fluid = false;
};

struct Mesh {
  std::vector<V3> X;
  std::vector<int64_t> fptr{0};
  std::vector<int32_t> fvert;
  std::vector<V3> fnormal;
  std::vector<std::array<int32_t, 2>> edges;
  std::vector<int64_t> cfptr{0};
  std::vector<int32_t> cface;
  std::vector<int8_t> corient;
  std::vector<int64_t> cvptr{0};
  std::vector<int32_t> cvert;
  std::vector<int64_t> ceptr{0};
  std::vector<int32_t> cedge;
  std::vector<double> cvol;
  std::vector<V3> ccen;
  std::vector<int32_t> ctile;
  std::vector<uint8_t> cplain;   // cell is an unsplit cube with unsplit faces
  std::vector<int32_t> cside;    // cube edge length in cells (plain cubes)
  int64_t nv() const { return static_cast<int64_t>(X.size()); }
  int64_t nf() const { return static_cast<int64_t>(fnormal.size()); }
  int64_t ne() const { return static_cast<int64_t>(edges.size()); }
  int64_t nc() const { return static_cast<int64_t>(cvol.size()); }
};

struct Level {
  std::vector<int8_t> E;                 // per background cell: cube exponent, -1 inside a cut tree
  std::vector<std::vector<uint8_t>> act; // per tree: node is an active cut
  std::vector<Tile> tiles;
  std::vector<int32_t> cube_tile;        // per background cell (cubes)
  std::vector<std::vector<int32_t>> tree_tiles;  // per tree: tiles of its current leaves
  Mesh mesh;
  // DOFs
  int64_t ndof = 0;          // all DOFs (vertices, edges, faces, cells)
  std::vector<int32_t> perm; // raw id -> ordered id
  std::vector<int32_t> free; // ordered id -> free index or -1
  int64_t nfree = 0;
};

inline int64_t bgi(int N, int i, int j, int k) { return (static_cast<int64_t>(i) * N + j) * N + k; }

}  // namespace

struct BuilderImpl {
  int N, k, L;
  double h;
  bool dirichlet;
  int64_t coarse_max;
  int max_levels;
  bool naive = false;
  std::vector<V3> TV;
  std::vector<std::array<int32_t, 3>> TF;
  std::vector<V3> tn;
  std::vector<double> td, tarea;
  double total_area = 0;
  std::vector<int32_t> tree_of;
  std::vector<Tree> trees;
  std::vector<int64_t> tri_cells;                // background cells with boundary triangles
  std::vector<std::vector<int32_t>> tri_lists;   // their triangles
  std::vector<uint8_t> bg_fluid;
  std::vector<Level> levels;
  std::vector<std::vector<int32_t>> parents;   // per level: fine cell -> coarse cell
  Output *out = nullptr;

  // ------------------------------------------------------------------ BSP
  void associate(std::vector<std::vector<int32_t>> &cell_tris, std::vector<int64_t> &cells) {
    const int nt = static_cast<int>(TF.size());
    std::vector<std::vector<std::pair<int64_t, int32_t>>> loc(omp_get_max_threads());
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < nt; ++t) {
      auto &L = loc[omp_get_thread_num()];
      const V3 a = TV[TF[t][0]], b = TV[TF[t][1]], c = TV[TF[t][2]];
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        const double mn = std::min({a[d], b[d], c[d]}), mx = std::max({a[d], b[d], c[d]});
        lo[d] = std::clamp(static_cast<int>(std::floor(mn / h - 1e-9)), 0, N - 1);
        hi[d] = std::clamp(static_cast<int>(std::floor(mx / h + 1e-9)), 0, N - 1);
      }
      for (int i = lo[0]; i <= hi[0]; ++i)
        for (int j = lo[1]; j <= hi[1]; ++j)
          for (int kk = lo[2]; kk <= hi[2]; ++kk) {
            const V3 blo(i * h, j * h, kk * h), bhi((i + 1) * h, (j + 1) * h, (kk + 1) * h);
            if (geo::tri_box_overlap(a, b, c, blo, bhi)) L.push_back({bgi(N, i, j, kk), t});
          }
    }
    std::vector<std::pair<int64_t, int32_t>> all;
    for (auto &l : loc) all.insert(all.end(), l.begin(), l.end());
    std::sort(all.begin(), all.end());
    for (size_t q = 0; q < all.size();) {
      size_t r = q;
      cells.push_back(all[q].first);
      cell_tris.emplace_back();
      while (r < all.size() && all[r].first == all[q].first) cell_tris.back().push_back(all[r++].second);
      q = r;
    }
  }

  bool tri_in(int32_t t, const Polyhedron &C) const {
    geo::Polygon P = {TV[TF[t][0]], TV[TF[t][1]], TV[TF[t][2]]};
    P = geo::clip_to(P, C);
    return P.size() >= 3 && geo::area(P) > 1e-14 * h * h;
  }

  bool coplanar(int32_t s, int32_t t) const {
    for (int v = 0; v < 3; ++v)
      if (std::fabs(dot(tn[t], TV[TF[s][v]]) - td[t]) > kPlaneTol) return false;
    return true;
  }

  Tree build_tree(int64_t bg, const std::vector<int32_t> &tris) const {
    Tree T;
    T.bg = bg;
    const int i = static_cast<int>(bg / (static_cast<int64_t>(N) * N));
    const int j = static_cast<int>((bg / N) % N), kk = static_cast<int>(bg % N);
    Node root;
    root.poly = geo::box(V3(i * h, j * h, kk * h), V3((i + 1) * h, (j + 1) * h, (kk + 1) * h));
    geo::volume_centroid(root.poly, &root.vol, &root.cen);
    T.nodes.push_back(root);
    // order: fewest crossings first
    std::vector<std::pair<int, int32_t>> ord;
    for (int32_t t : tris) {
      int cnt = 0;
      for (int32_t s : tris) {
        if (s == t) continue;
        double mn = 1e300, mx = -1e300;
        for (int v = 0; v < 3; ++v) {
          const double sd = dot(tn[t], TV[TF[s][v]]) - td[t];
          mn = std::min(mn, sd);
          mx = std::max(mx, sd);
        }
        if (mx > kPlaneTol && mn < -kPlaneTol) ++cnt;
      }
      ord.push_back({cnt, t});
    }
    std::sort(ord.begin(), ord.end());
    std::vector<int32_t> order;
    for (auto &o : ord) order.push_back(o.second);
    std::vector<std::pair<int, std::vector<int32_t>>> stack;
    stack.push_back({0, order});
    while (!stack.empty()) {
      auto [nid, pending] = std::move(stack.back());
      stack.pop_back();
      size_t q = 0;
      while (q < pending.size()) {
        const int32_t t = pending[q];
        Polyhedron below, above;
        const bool cut = geo::split(T.nodes[nid].poly, tn[t], td[t], &below, &above);
        double vb = 0, va = 0;
        V3 cb, ca;
        if (cut) {
          geo::volume_centroid(below, &vb, &cb);
          geo::volume_centroid(above, &va, &ca);
        }
        // remaining list without t and the triangles coplanar with it
        std::vector<int32_t> rest, cop;
        for (size_t r = q; r < pending.size(); ++r) {
          const int32_t s = pending[r];
          if (s == t || coplanar(s, t)) cop.push_back(s);
          else rest.push_back(s);
        }
        if (!cut || vb < kMinVolume || va < kMinVolume) {
          pending = std::move(rest);
          q = 0;
          continue;
        }
        double covered = 0;
        for (int32_t s : cop) {
          geo::Polygon P = {TV[TF[s][0]], TV[TF[s][1]], TV[TF[s][2]]};
          P = geo::clip_to(P, T.nodes[nid].poly);
          if (P.size() >= 3) covered += geo::area(P);
        }
        Node &nd = T.nodes[nid];
        nd.n = tn[t];
        nd.d = td[t];
        nd.w = covered / total_area;
        Node c0, c1;
        c0.poly = std::move(below);
        c0.vol = vb;
        c0.cen = cb;
        c0.parent = nid;
        c1.poly = std::move(above);
        c1.vol = va;
        c1.cen = ca;
        c1.parent = nid;
        const int id0 = static_cast<int>(T.nodes.size());
        T.nodes.push_back(std::move(c0));
        T.nodes.push_back(std::move(c1));
        T.nodes[nid].child[0] = id0;
        T.nodes[nid].child[1] = id0 + 1;
        for (int side = 1; side >= 0; --side) {
          std::vector<int32_t> sub;
          for (int32_t s : rest)
            if (tri_in(s, T.nodes[id0 + side].poly)) sub.push_back(s);
          stack.push_back({id0 + side, std::move(sub)});
        }
        break;
      }
    }
    return T;
  }

  void build_forest() {
    associate(tri_lists, tri_cells);
    const std::vector<std::vector<int32_t>> &cell_tris = tri_lists;
    const std::vector<int64_t> &cells = tri_cells;
    std::vector<Tree> all(cells.size());
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < static_cast<int64_t>(cells.size()); ++q) all[q] = build_tree(cells[q], cell_tris[q]);
    const int64_t N3 = static_cast<int64_t>(N) * N * N;
    tree_of.assign(N3, -1);
    for (auto &T : all)
      if (T.nodes.size() > 1) {
        tree_of[T.bg] = static_cast<int32_t>(trees.size());
        trees.push_back(std::move(T));
      }
    // classification
    geo::Winding wind(TV, TF, N);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < static_cast<int64_t>(trees.size()); ++q) {
      auto &nodes = trees[q].nodes;
      for (auto &nd : nodes)
        if (nd.child[0] < 0) nd.fluid = wind.at(nd.cen) <= 0;
      for (int64_t a = static_cast<int64_t>(nodes.size()) - 1; a >= 0; --a)
        if (nodes[a].child[0] >= 0) nodes[a].fluid = nodes[nodes[a].child[0]].fluid || nodes[nodes[a].child[1]].fluid;
    }
    bg_fluid.assign(N3, 0);
    std::vector<uint8_t> has_tri(N3, 0);
    for (int64_t c : cells) has_tri[c] = 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int ij = 0; ij < N * N; ++ij) {
      const int i = ij / N, j = ij % N;
      int prev = -1;   // classification of the cell above if it had no triangles
      for (int kk = N - 1; kk >= 0; --kk) {
        const int64_t b = bgi(N, i, j, kk);
        if (tree_of[b] >= 0) {
          bg_fluid[b] = trees[tree_of[b]].nodes[0].fluid;
          prev = -1;
          continue;
        }
        if (has_tri[b] || prev < 0) {
          const V3 c((i + 0.5) * h, (j + 0.5) * h, (kk + 0.5) * h);
          bg_fluid[b] = wind.at(c) <= 0;
        } else {
          bg_fluid[b] = static_cast<uint8_t>(prev);
        }
        prev = has_tri[b] ? -1 : bg_fluid[b];
      }
    }
  }

  // ------------------------------------------------------------------ levels
  Level initial_level() {
    Level lv;
    const int64_t N3 = static_cast<int64_t>(N) * N * N;
    lv.E.assign(N3, 0);
    lv.act.resize(trees.size());
    for (size_t t = 0; t < trees.size(); ++t) {
      lv.E[trees[t].bg] = -1;
      lv.act[t].assign(trees[t].nodes.size(), 0);
      for (size_t a = 0; a < trees[t].nodes.size(); ++a) lv.act[t][a] = trees[t].nodes[a].child[0] >= 0;
    }
    return lv;
  }

  std::vector<int32_t> leaves(const Level &lv, int t) const {
    std::vector<int32_t> out, st{0};
    const auto &nodes = trees[t].nodes;
    while (!st.empty()) {
      const int a = st.back();
      st.pop_back();
      if (lv.act[t][a]) {
        st.push_back(nodes[a].child[1]);
        st.push_back(nodes[a].child[0]);
      } else {
        out.push_back(a);
      }
    }
    std::sort(out.begin(), out.end());
    return out;
  }

  void make_tiles(Level &lv) {
    const int64_t N3 = static_cast<int64_t>(N) * N * N;
    lv.tiles.clear();
    lv.cube_tile.assign(N3, -1);
    lv.tree_tiles.assign(trees.size(), {});
    for (size_t t = 0; t < trees.size(); ++t) {
      if (lv.E[trees[t].bg] >= 0) continue;
      const int64_t b = trees[t].bg;
      const int i = static_cast<int>(b / (static_cast<int64_t>(N) * N)), j = static_cast<int>((b / N) % N),
                kk = static_cast<int>(b % N);
      for (int32_t a : leaves(lv, static_cast<int>(t))) {
        Tile T;
        T.type = 0;
        T.tree = static_cast<int32_t>(t);
        T.node = a;
        T.lo[0] = i, T.lo[1] = j, T.lo[2] = kk;
        T.hi[0] = i + 1, T.hi[1] = j + 1, T.hi[2] = kk + 1;
        T.fluid = trees[t].nodes[a].fluid;
        lv.tree_tiles[t].push_back(static_cast<int32_t>(lv.tiles.size()));
        lv.tiles.push_back(T);
      }
    }
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        for (int kk = 0; kk < N; ++kk) {
          const int64_t b = bgi(N, i, j, kk);
          const int s = lv.E[b];
          if (s < 0 || lv.cube_tile[b] >= 0) continue;
          const int w = 1 << s;
          Tile T;
          T.type = 1;
          T.s = s;
          T.lo[0] = i - i % w, T.lo[1] = j - j % w, T.lo[2] = kk - kk % w;
          for (int d = 0; d < 3; ++d) T.hi[d] = T.lo[d] + w;
          bool fl = false;
          const int32_t id = static_cast<int32_t>(lv.tiles.size());
          for (int a = T.lo[0]; a < T.hi[0]; ++a)
            for (int bb = T.lo[1]; bb < T.hi[1]; ++bb)
              for (int c = T.lo[2]; c < T.hi[2]; ++c) {
                const int64_t q = bgi(N, a, bb, c);
                lv.cube_tile[q] = id;
                fl = fl || bg_fluid[q];
              }
          T.fluid = fl;
          lv.tiles.push_back(T);
        }
  }

  Polyhedron tile_poly(const Tile &T) const {
    if (T.type == 0) return trees[T.tree].nodes[T.node].poly;
    return geo::box(V3(T.lo[0] * h, T.lo[1] * h, T.lo[2] * h), V3(T.hi[0] * h, T.hi[1] * h, T.hi[2] * h));
  }

  Level coarsen(const Level &f, bool *changed) {
    Level c;
    c.E = f.E;
    c.act = f.act;
    const int64_t N3 = static_cast<int64_t>(N) * N * N;
    // balanced aggregation against the state at the start of the pass
    int smax = 0;
    for (int64_t q = 0; q < N3; ++q) smax = std::max(smax, static_cast<int>(f.E[q]));
    int merged = 0;
    for (int s = 0; s <= smax; ++s) {
      const int w = 1 << (s + 1);
      if (w > N) break;
      const int nb = N / w;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : merged)
      for (int64_t blk = 0; blk < static_cast<int64_t>(nb) * nb * nb; ++blk) {
        const int bi = static_cast<int>(blk / (static_cast<int64_t>(nb) * nb)) * w;
        const int bj = static_cast<int>((blk / nb) % nb) * w, bk = static_cast<int>(blk % nb) * w;
        bool ok = true;
        for (int a = bi; a < bi + w && ok; ++a)
          for (int b = bj; b < bj + w && ok; ++b)
            for (int cc = bk; cc < bk + w && ok; ++cc)
              if (f.E[bgi(N, a, b, cc)] != s) ok = false;
        if (!ok) continue;
        for (int a = std::max(bi - 1, 0); a < std::min(bi + w + 1, N) && ok; ++a)
          for (int b = std::max(bj - 1, 0); b < std::min(bj + w + 1, N) && ok; ++b)
            for (int cc = std::max(bk - 1, 0); cc < std::min(bk + w + 1, N) && ok; ++cc) {
              const int e = f.E[bgi(N, a, b, cc)];
              if ((e < 0 ? 0 : e) < s) ok = false;
            }
        if (!ok) continue;
        for (int a = bi; a < bi + w; ++a)
          for (int b = bj; b < bj + w; ++b)
            for (int cc = bk; cc < bk + w; ++cc) c.E[bgi(N, a, b, cc)] = static_cast<int8_t>(s + 1);
        ++merged;
      }
    }
    // greedy removal of the least important removable cuts
    using Key = std::tuple<double, int64_t, int32_t, int32_t>;   // weight, bg, node, tree
    std::priority_queue<Key, std::vector<Key>, std::greater<Key>> pq;
    auto removable = [&](int t, int a) {
      const auto &nd = trees[t].nodes[a];
      return c.act[t][a] && !c.act[t][nd.child[0]] && !c.act[t][nd.child[1]];
    };
    for (size_t t = 0; t < trees.size(); ++t)
      for (size_t a = 0; a < trees[t].nodes.size(); ++a)
        if (removable(static_cast<int>(t), static_cast<int>(a)))
          pq.push({trees[t].nodes[a].w, trees[t].bg, static_cast<int32_t>(a), static_cast<int32_t>(t)});
    double removed = 0;
    int nrem = 0;
    while (!pq.empty() && removed <= 1.0 / L) {
      const auto [w, bg, a, t] = pq.top();
      pq.pop();
      c.act[t][a] = 0;
      removed += w;
      ++nrem;
      const int par = trees[t].nodes[a].parent;
      if (par >= 0 && removable(t, par)) pq.push({trees[t].nodes[par].w, bg, par, t});
      bool any = false;
      for (uint8_t v : c.act[t]) any = any || v;
      if (!any) c.E[bg] = 0;
    }
    *changed = merged > 0 || nrem > 0;
    return c;
  }

  // ------------------------------------------------------------------ conforming mesh
  struct Pool {
    double h;
    int N;
    std::vector<int32_t> lattice;
    std::unordered_map<uint64_t, std::vector<int32_t>> hash;
    std::vector<V3> X;
    int32_t get(V3 p) {
      const double gi = p.x / h, gj = p.y / h, gk = p.z / h;
      const double ri = std::nearbyint(gi), rj = std::nearbyint(gj), rk = std::nearbyint(gk);
      if (std::fabs(gi - ri) * h < kVertTol && std::fabs(gj - rj) * h < kVertTol && std::fabs(gk - rk) * h < kVertTol) {
        const int64_t key = (static_cast<int64_t>(ri) * (N + 1) + static_cast<int64_t>(rj)) * (N + 1) + static_cast<int64_t>(rk);
        int32_t &v = lattice[key];
        if (v < 0) {
          v = static_cast<int32_t>(X.size());
          X.push_back(V3(ri * h, rj * h, rk * h));
        }
        return v;
      }
      const double q = kVertTol;   // bucket width: a weld partner lies in a neighbouring bucket
      const int64_t bx = static_cast<int64_t>(std::floor(p.x / q)), by = static_cast<int64_t>(std::floor(p.y / q)),
                    bz = static_cast<int64_t>(std::floor(p.z / q));
      auto key = [](int64_t a, int64_t b, int64_t c) {
        return static_cast<uint64_t>(a) * 0x9E3779B97F4A7C15ULL ^ static_cast<uint64_t>(b) * 0xC2B2AE3D27D4EB4FULL ^
               static_cast<uint64_t>(c) * 0x165667B19E3779F9ULL;
      };
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            auto it = hash.find(key(bx + dx, by + dy, bz + dz));
            if (it == hash.end()) continue;
            for (int32_t v : it->second)
              if (norm(X[v] - p) < kVertTol) return v;
          }
      const int32_t v = static_cast<int32_t>(X.size());
      X.push_back(p);
      hash[key(bx, by, bz)].push_back(v);
      return v;
    }
  };

  void conform(Level &lv) {
    const auto &tiles = lv.tiles;
    const int64_t nt = static_cast<int64_t>(tiles.size());
    std::vector<int32_t> fl;
    for (int64_t t = 0; t < nt; ++t)
      if (tiles[t].fluid) fl.push_back(static_cast<int32_t>(t));
    const int64_t nc = static_cast<int64_t>(fl.size());
    std::vector<uint8_t> plain(nc, 0);
    std::vector<std::vector<geo::Polygon>> pieces(nc);
    std::vector<std::vector<V3>> piece_n(nc);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : bad)
    for (int64_t ci = 0; ci < nc; ++ci) {
      const Tile &T = tiles[fl[ci]];
      std::vector<int32_t> neigh;
      bool is_plain = T.type == 1;
      for (int a = std::max(T.lo[0] - 1, 0); a < std::min(T.hi[0] + 1, N); ++a)
        for (int b = std::max(T.lo[1] - 1, 0); b < std::min(T.hi[1] + 1, N); ++b)
          for (int c = std::max(T.lo[2] - 1, 0); c < std::min(T.hi[2] + 1, N); ++c) {
            const int64_t q = bgi(N, a, b, c);
            if (lv.cube_tile[q] >= 0) {
              neigh.push_back(lv.cube_tile[q]);
              if (tiles[lv.cube_tile[q]].s != T.s) is_plain = false;
            } else {
              is_plain = false;
              const auto &tt = lv.tree_tiles[tree_of[q]];
              neigh.insert(neigh.end(), tt.begin(), tt.end());
            }
          }
      plain[ci] = is_plain;
      const Polyhedron P = tile_poly(T);
      if (is_plain) {
        for (const auto &f : P) {
          pieces[ci].push_back(f.p);
          piece_n[ci].push_back(f.n);
        }
        continue;
      }
      std::sort(neigh.begin(), neigh.end());
      neigh.erase(std::unique(neigh.begin(), neigh.end()), neigh.end());
      std::vector<Polyhedron> npoly;
      for (int32_t g : neigh)
        if (g != fl[ci]) npoly.push_back(tile_poly(tiles[g]));
      for (const auto &f : P) {
        std::vector<geo::Polygon> got;
        for (const auto &Q : npoly)
          for (const auto &g : Q) {
            if (std::fabs(f.n.x + g.n.x) + std::fabs(f.n.y + g.n.y) + std::fabs(f.n.z + g.n.z) >= 1e-9) continue;
            if (std::fabs(f.d + g.d) >= 1e-9) continue;
            geo::Polygon O = geo::overlap(f.p, g.p, g.n);
            if (O.size() < 3) continue;
            double per = 0;
            for (size_t i = 0; i < O.size(); ++i) per += norm(O[(i + 1) % O.size()] - O[i]);
            if (per <= 0 || 2.0 * geo::area(O) / per <= 1e-11) continue;
            got.push_back(std::move(O));
          }
        if (got.empty()) {
          got.push_back(f.p);
        } else {
          double s = 0;
          for (auto &O : got) s += geo::area(O);
          const double ap = geo::area(f.p);
          if (std::fabs(s - ap) > 1e-9 * std::max(ap, h * h)) bad = 1;
        }
        for (auto &O : got) {
          pieces[ci].push_back(std::move(O));
          piece_n[ci].push_back(f.n);
        }
      }
    }
    if (bad) throw std::runtime_error("facet overlay does not cover a facet");
    // vertex ids (sequential: deterministic)
    Pool pool;
    pool.h = h;
    pool.N = N;
    pool.lattice.assign(static_cast<size_t>(N + 1) * (N + 1) * (N + 1), -1);
    std::vector<std::vector<std::vector<int32_t>>> cyc(nc);
    for (int64_t ci = 0; ci < nc; ++ci) {
      for (auto &P : pieces[ci]) {
        std::vector<int32_t> ids;
        for (const V3 &p : P) {
          const int32_t v = pool.get(p);
          if (ids.empty() || ids.back() != v) ids.push_back(v);
        }
        while (ids.size() > 1 && ids.front() == ids.back()) ids.pop_back();
        if (ids.size() >= 3) cyc[ci].push_back(std::move(ids));
      }
      std::vector<geo::Polygon>().swap(pieces[ci]);
    }
    Mesh &M = lv.mesh;
    M = Mesh();
    M.X = std::move(pool.X);
    // T-junctions
    const double hb = 0.5 * h;
    std::unordered_map<uint64_t, std::vector<int32_t>> bucket;
    auto bkey = [](int64_t a, int64_t b, int64_t c) {
      return (static_cast<uint64_t>(a + 4) << 42) | (static_cast<uint64_t>(b + 4) << 21) | static_cast<uint64_t>(c + 4);
    };
    for (int32_t v = 0; v < static_cast<int32_t>(M.X.size()); ++v)
      bucket[bkey(static_cast<int64_t>(std::floor(M.X[v].x / hb)), static_cast<int64_t>(std::floor(M.X[v].y / hb)),
                  static_cast<int64_t>(std::floor(M.X[v].z / hb)))]
          .push_back(v);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t ci = 0; ci < nc; ++ci) {
      if (plain[ci]) continue;
      for (auto &cy : cyc[ci]) {
        std::vector<int32_t> nw;
        const size_t m = cy.size();
        for (size_t i = 0; i < m; ++i) {
          const int32_t a = cy[i], b = cy[(i + 1) % m];
          nw.push_back(a);
          const V3 pa = M.X[a], pb = M.X[b], ab = pb - pa;
          const double L2 = dot(ab, ab);
          int64_t lo[3], hi[3];
          for (int d = 0; d < 3; ++d) {
            lo[d] = static_cast<int64_t>(std::floor((std::min(pa[d], pb[d]) - 1e-9) / hb));
            hi[d] = static_cast<int64_t>(std::floor((std::max(pa[d], pb[d]) + 1e-9) / hb));
          }
          std::vector<std::pair<double, int32_t>> found;
          for (int64_t x = lo[0]; x <= hi[0]; ++x)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
              for (int64_t z = lo[2]; z <= hi[2]; ++z) {
                auto it = bucket.find(bkey(x, y, z));
                if (it == bucket.end()) continue;
                for (int32_t v : it->second) {
                  if (v == a || v == b) continue;
                  const V3 w = M.X[v] - pa;
                  const double tau = dot(w, ab) / L2;
                  if (tau <= 1e-12 || tau >= 1 - 1e-12) continue;
                  if (norm(w - tau * ab) < kVertTol) found.push_back({tau, v});
                }
              }
          std::sort(found.begin(), found.end());
          for (auto &fv : found) nw.push_back(fv.second);
        }
        cy = std::move(nw);
      }
    }
    // faces and edges, numbered in cell order (deterministic).  Per chunk of
    // cells, each cycle's sorted vertex list, hash and unit normal are formed
    // in parallel; the numbering itself is a sequential pass over flat maps.
    FlatMap fhead(static_cast<size_t>(4 * nc + 16));   // cycle hash -> newest face with that hash
    // edges by their lower vertex: a few inline (upper vertex, edge) slots
    // per vertex, which neighbouring cells reach in nearby memory, and a
    // map for vertices with more edges than slots
    constexpr int EDGE_SLOTS = 6;
    std::vector<std::array<int32_t, 2 * EDGE_SLOTS>> vadj(M.X.size());
    for (auto &sl : vadj) sl.fill(-1);
    FlatMap emap(1024);
    std::vector<int32_t> fnext;                         // older face with the same hash, or -1
    std::vector<int32_t> fkey;                          // sorted vertex ids per face (offsets M.fptr)
    M.ctile.resize(nc);
    M.cplain.resize(nc);
    M.cside.resize(nc);
    constexpr int64_t CHUNK = 65536;
    std::vector<int64_t> cbeg, kbeg;
    std::vector<int32_t> kbuf;
    std::vector<uint64_t> hbuf;
    std::vector<V3> nbuf;
    for (int64_t c0 = 0; c0 < nc; c0 += CHUNK) {
      const int64_t c1 = std::min(nc, c0 + CHUNK);
      cbeg.assign(c1 - c0 + 1, 0);
      for (int64_t ci = c0; ci < c1; ++ci) cbeg[ci - c0 + 1] = cbeg[ci - c0] + static_cast<int64_t>(cyc[ci].size());
      const int64_t ncy = cbeg.back();
      kbeg.assign(ncy + 1, 0);
      {
        int64_t q = 0;
        for (int64_t ci = c0; ci < c1; ++ci)
          for (auto &cy : cyc[ci]) {
            kbeg[q + 1] = kbeg[q] + static_cast<int64_t>(cy.size());
            ++q;
          }
      }
      kbuf.resize(kbeg[ncy]);
      hbuf.resize(ncy);
      nbuf.resize(ncy);
#pragma omp parallel for schedule(dynamic, 256)
      for (int64_t ci = c0; ci < c1; ++ci) {
        std::vector<V3> P;
        int64_t q = cbeg[ci - c0];
        for (auto &cy : cyc[ci]) {
          int32_t *key = kbuf.data() + kbeg[q];
          std::copy(cy.begin(), cy.end(), key);
          std::sort(key, key + cy.size());
          uint64_t hk = 1469598103934665603ULL;
          for (size_t t = 0; t < cy.size(); ++t) hk = (hk ^ static_cast<uint64_t>(key[t])) * 1099511628211ULL;
          hbuf[q] = hk == FlatMap::EMPTY ? hk - 1 : hk;
          P.clear();
          for (int32_t v : cy) P.push_back(M.X[v]);
          const V3 nvec = geo::area_vector(P);
          nbuf[q] = (1.0 / norm(nvec)) * nvec;
          ++q;
        }
      }
      int64_t q = 0;
      for (int64_t ci = c0; ci < c1; ++ci) {
        M.ctile[ci] = fl[ci];
        M.cplain[ci] = plain[ci];
        M.cside[ci] = tiles[fl[ci]].type == 1 ? (1 << tiles[fl[ci]].s) : 0;
        std::vector<int32_t> lv_verts, lv_edges;
        for (auto &cy : cyc[ci]) {
          const int32_t *key = kbuf.data() + kbeg[q];
          const int64_t m = static_cast<int64_t>(cy.size());
          const V3 nvec = nbuf[q];
          bool fresh;
          int32_t *head = fhead.find_or_insert(hbuf[q], &fresh);
          int32_t fid = -1;
          if (!fresh)
            for (int32_t f = *head; f >= 0; f = fnext[f])
              if (M.fptr[f + 1] - M.fptr[f] == m && std::equal(key, key + m, fkey.begin() + M.fptr[f])) {
                fid = f;
                break;
              }
          if (fid < 0) {
            fid = static_cast<int32_t>(M.fnormal.size());
            fnext.push_back(fresh ? -1 : *head);
            *head = fid;
            M.fvert.insert(M.fvert.end(), cy.begin(), cy.end());
            fkey.insert(fkey.end(), key, key + m);
            M.fptr.push_back(static_cast<int64_t>(M.fvert.size()));
            M.fnormal.push_back(nvec);
            M.cface.push_back(fid);
            M.corient.push_back(1);
          } else {
            M.cface.push_back(fid);
            M.corient.push_back(dot(M.fnormal[fid], nvec) > 0 ? 1 : -1);
          }
          for (int64_t i = 0; i < m; ++i) {
            const int32_t a = cy[i], b = cy[(i + 1) % m];
            if (std::find(lv_verts.begin(), lv_verts.end(), a) == lv_verts.end()) lv_verts.push_back(a);
            const uint64_t ek = (static_cast<uint64_t>(std::min(a, b)) << 32) | static_cast<uint32_t>(std::max(a, b));
            const int32_t lo = std::min(a, b), hi = std::max(a, b);
            int32_t e = -1;
            auto &sl = vadj[lo];
            int t = 0;
            for (; t < EDGE_SLOTS && sl[2 * t] >= 0; ++t)
              if (sl[2 * t] == hi) {
                e = sl[2 * t + 1];
                break;
              }
            if (e < 0) {
              int32_t *slot = nullptr;
              bool fresh_e = true;
              if (t == EDGE_SLOTS) slot = emap.find_or_insert(ek, &fresh_e);
              if (fresh_e) {
                e = static_cast<int32_t>(M.edges.size());
                M.edges.push_back({lo, hi});
                if (slot) *slot = e;
                else {
                  sl[2 * t] = hi;
                  sl[2 * t + 1] = e;
                }
              } else {
                e = *slot;
              }
            }
            if (std::find(lv_edges.begin(), lv_edges.end(), e) == lv_edges.end()) lv_edges.push_back(e);
          }
          ++q;
        }
        M.cfptr.push_back(static_cast<int64_t>(M.cface.size()));
        M.cvert.insert(M.cvert.end(), lv_verts.begin(), lv_verts.end());
        M.cvptr.push_back(static_cast<int64_t>(M.cvert.size()));
        M.cedge.insert(M.cedge.end(), lv_edges.begin(), lv_edges.end());
        M.ceptr.push_back(static_cast<int64_t>(M.cedge.size()));
        std::vector<std::vector<int32_t>>().swap(cyc[ci]);
      }
    }
    M.cvol.resize(nc);
    M.ccen.resize(nc);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t ci = 0; ci < nc; ++ci) {
      Polyhedron C;
      for (int64_t q = M.cfptr[ci]; q < M.cfptr[ci + 1]; ++q) {
        geo::Facet f;
        f.p = face_points(M, M.cface[q], M.corient[q]);
        C.push_back(f);
      }
      geo::volume_centroid(C, &M.cvol[ci], &M.ccen[ci]);
    }
  }

  static std::vector<V3> face_points(const Mesh &M, int32_t f, int8_t o) {
    std::vector<V3> P;
    for (int64_t q = M.fptr[f]; q < M.fptr[f + 1]; ++q) P.push_back(M.X[M.fvert[q]]);
    if (o < 0) std::reverse(P.begin(), P.end());
    return P;
  }

  // local VEM cell of mesh cell c
  vem::Cell vem_cell(const Mesh &M, int64_t c) const {
    vem::Cell C;
    std::unordered_map<int32_t, int> vl, el;
    for (int64_t q = M.cvptr[c]; q < M.cvptr[c + 1]; ++q) {
      vl[M.cvert[q]] = static_cast<int>(C.X.size());
      C.X.push_back(M.X[M.cvert[q]]);
    }
    for (int64_t q = M.ceptr[c]; q < M.ceptr[c + 1]; ++q) {
      const auto &e = M.edges[M.cedge[q]];
      el[M.cedge[q]] = static_cast<int>(C.edges.size());
      C.edges.push_back({vl[e[0]], vl[e[1]]});
    }
    for (int64_t q = M.cfptr[c]; q < M.cfptr[c + 1]; ++q) {
      const int32_t f = M.cface[q];
      std::vector<int32_t> gv(M.fvert.begin() + M.fptr[f], M.fvert.begin() + M.fptr[f + 1]);
      if (M.corient[q] < 0) std::reverse(gv.begin(), gv.end());
      std::vector<int> lc, le;
      for (size_t i = 0; i < gv.size(); ++i) {
        lc.push_back(vl[gv[i]]);
        const int32_t a = gv[i], b = gv[(i + 1) % gv.size()];
        le.push_back(-1);
        for (int64_t r = M.ceptr[c]; r < M.ceptr[c + 1]; ++r) {
          const auto &e = M.edges[M.cedge[r]];
          if ((e[0] == a && e[1] == b) || (e[0] == b && e[1] == a)) {
            le.back() = el[M.cedge[r]];
            break;
          }
        }
      }
      C.faces.push_back(lc);
      C.face_edges.push_back(le);
    }
    return C;
  }

  // ------------------------------------------------------------------ DOFs
  // raw DOF ids: vertices, then (k = 2) edges, faces, cells
  int64_t raw_count(const Mesh &M) const { return k == 1 ? M.nv() : M.nv() + M.ne() + M.nf() + M.nc(); }

  std::vector<int32_t> cell_raw_dofs(const Mesh &M, int64_t c) const {
    std::vector<int32_t> d(M.cvert.begin() + M.cvptr[c], M.cvert.begin() + M.cvptr[c + 1]);
    if (k == 2) {
      for (int64_t q = M.ceptr[c]; q < M.ceptr[c + 1]; ++q) d.push_back(static_cast<int32_t>(M.nv() + M.cedge[q]));
      for (int64_t q = M.cfptr[c]; q < M.cfptr[c + 1]; ++q)
        d.push_back(static_cast<int32_t>(M.nv() + M.ne() + M.cface[q]));
      d.push_back(static_cast<int32_t>(M.nv() + M.ne() + M.nf() + c));
    }
    return d;
  }

  static uint64_t morton(uint32_t i, uint32_t j, uint32_t kk) {
    uint64_t m = 0;
    for (int b = 0; b < 10; ++b)
      m |= ((static_cast<uint64_t>(i >> b) & 1) << (3 * b + 2)) | ((static_cast<uint64_t>(j >> b) & 1) << (3 * b + 1)) |
           ((static_cast<uint64_t>(kk >> b) & 1) << (3 * b));
    return m;
  }

  V3 raw_point(const Mesh &M, int64_t r) const {
    if (r < M.nv()) return M.X[r];
    r -= M.nv();
    if (r < M.ne()) return 0.5 * (M.X[M.edges[r][0]] + M.X[M.edges[r][1]]);
    r -= M.ne();
    if (r < M.nf()) {
      V3 c;
      for (int64_t q = M.fptr[r]; q < M.fptr[r + 1]; ++q) c = c + M.X[M.fvert[q]];
      return (1.0 / static_cast<double>(M.fptr[r + 1] - M.fptr[r])) * c;
    }
    return M.ccen[r - M.nf()];
  }

  int raw_kind(const Mesh &M, int64_t r) const {
    if (r < M.nv()) return 0;
    if (r < M.nv() + M.ne()) return 1;
    if (r < M.nv() + M.ne() + M.nf()) return 2;
    return 3;
  }

  // spatially ordered numbering (4^3-cell tiles in Morton order, by DOF kind inside a tile)
  void number_dofs(Level &lv) {
    const Mesh &M = lv.mesh;
    const int64_t n = raw_count(M);
    lv.ndof = n;
    std::vector<std::pair<std::array<uint64_t, 2>, int32_t>> key(n);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
      const V3 p = raw_point(M, r);
      const uint32_t i = static_cast<uint32_t>(std::clamp(static_cast<int>(p.x / h), 0, N - 1));
      const uint32_t j = static_cast<uint32_t>(std::clamp(static_cast<int>(p.y / h), 0, N - 1));
      const uint32_t kk = static_cast<uint32_t>(std::clamp(static_cast<int>(p.z / h), 0, N - 1));
      const uint64_t mo = morton(i, j, kk);
      key[r] = {{((mo >> 6) << 2) | static_cast<uint64_t>(raw_kind(M, r)), mo}, static_cast<int32_t>(r)};
    }
    // keys are unique (they end in the raw id), so the parallel sort gives
    // the serial order
    __gnu_parallel::sort(key.begin(), key.end());
    lv.perm.assign(n, -1);
    for (int64_t q = 0; q < n; ++q) lv.perm[key[q].second] = static_cast<int32_t>(q);
    // Dirichlet: DOFs supported on z = 1
    std::vector<uint8_t> dir(n, 0);
    if (dirichlet) {
      std::vector<uint8_t> top(M.nv());
      for (int64_t v = 0; v < M.nv(); ++v) top[v] = std::fabs(M.X[v].z - 1.0) < 1e-12;
      for (int64_t v = 0; v < M.nv(); ++v) dir[v] = top[v];
      if (k == 2) {
        for (int64_t e = 0; e < M.ne(); ++e) dir[M.nv() + e] = top[M.edges[e][0]] && top[M.edges[e][1]];
        for (int64_t f = 0; f < M.nf(); ++f) {
          bool all = true;
          for (int64_t q = M.fptr[f]; q < M.fptr[f + 1]; ++q) all = all && top[M.fvert[q]];
          dir[M.nv() + M.ne() + f] = all;
        }
      }
    }
    lv.free.assign(n, -1);
    std::vector<uint8_t> dir_ord(n);
    for (int64_t r = 0; r < n; ++r) dir_ord[lv.perm[r]] = dir[r];
    int64_t nf = 0;
    for (int64_t q = 0; q < n; ++q)
      if (!dir_ord[q]) lv.free[q] = static_cast<int32_t>(nf++);
    lv.nfree = nf;
  }

  void drop_unused(Level &lv, const std::vector<uint8_t> &used_free) {
    int64_t nf = 0;
    for (int64_t q = 0; q < lv.ndof; ++q) {
      if (lv.free[q] < 0) continue;
      lv.free[q] = used_free[lv.free[q]] ? static_cast<int32_t>(nf++) : -1;
    }
    lv.nfree = nf;
  }

  // ------------------------------------------------------------------ prolongation
  struct Row {
    std::vector<std::pair<int32_t, double>> e;   // (coarse raw DOF, weight)
  };

  void prolongation(int l, std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<double> &va) {
    Level &F = levels[l], &C = levels[l + 1];
    const Mesh &Mf = F.mesh, &Mc = C.mesh;
    const auto &par = parents[l];
    const int64_t ncc = Mc.nc();
    // coarse projectors
    std::vector<vem::CellData> cproj(ncc);
    std::vector<vem::Cell> ccell(ncc);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < ncc; ++c) {
      ccell[c] = vem_cell(Mc, c);
      cproj[c] = vem::projector(ccell[c], k);
    }
    std::vector<vem::FaceProj> fproj(Mc.nf());
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t f = 0; f < Mc.nf(); ++f) fproj[f] = vem::face_projector(face_points(Mc, static_cast<int32_t>(f), 1), Mc.fnormal[f], k);
    auto face_raw = [&](int64_t f) {
      std::vector<int32_t> d(Mc.fvert.begin() + Mc.fptr[f], Mc.fvert.begin() + Mc.fptr[f + 1]);
      if (k == 2) {
        const size_t m = d.size();
        std::vector<int32_t> e;
        for (size_t i = 0; i < m; ++i) {
          const int32_t a = d[i], b = d[(i + 1) % m];
          int32_t eid = -1;
          // edge of the coarse face: search the cells' edge lists would be slow; use the edge map
          auto it = cedge_map.find((static_cast<uint64_t>(std::min(a, b)) << 32) | static_cast<uint32_t>(std::max(a, b)));
          if (it != cedge_map.end()) eid = it->second;
          e.push_back(static_cast<int32_t>(Mc.nv() + eid));
        }
        d.insert(d.end(), e.begin(), e.end());
        d.push_back(static_cast<int32_t>(Mc.nv() + Mc.ne() + f));
      }
      return d;
    };
    cedge_map.clear();
    for (int64_t e = 0; e < Mc.ne(); ++e)
      cedge_map[(static_cast<uint64_t>(Mc.edges[e][0]) << 32) | static_cast<uint32_t>(Mc.edges[e][1])] = static_cast<int32_t>(e);
    // owner of each fine raw DOF: first fine cell containing it
    const int64_t nrf = raw_count(Mf);
    std::vector<int32_t> owner(nrf, -1);
    for (int64_t c = 0; c < Mf.nc(); ++c)
      for (int32_t r : cell_raw_dofs(Mf, c))
        if (owner[r] < 0) owner[r] = static_cast<int32_t>(c);
    std::vector<Row> rows(nrf);
    constexpr double tol = 1e-9;
    // naive prolongation: coarse cells around each vertex, and whether a
    // point lies in a coarse cell's closure
    std::vector<std::vector<int32_t>> vcells;
    if (naive) {
      vcells.resize(Mc.nv());
      for (int64_t c = 0; c < ncc; ++c)
        for (int64_t q = Mc.cvptr[c]; q < Mc.cvptr[c + 1]; ++q) vcells[Mc.cvert[q]].push_back(static_cast<int32_t>(c));
    }
    auto in_cell = [&](int64_t c, V3 p) {
      for (int64_t q = Mc.cfptr[c]; q < Mc.cfptr[c + 1]; ++q) {
        const int32_t f = Mc.cface[q];
        const V3 n = static_cast<double>(Mc.corient[q]) * Mc.fnormal[f];
        if (dot(n, p - Mc.X[Mc.fvert[Mc.fptr[f]]]) > tol) return false;
      }
      return true;
    };
    // coarse cells (E first, then increasing id) whose closure holds all points
    auto cells_holding = [&](int32_t E, const std::vector<V3> &pts) {
      std::vector<int32_t> cand;
      for (int64_t q = Mc.cvptr[E]; q < Mc.cvptr[E + 1]; ++q)
        for (int32_t c : vcells[Mc.cvert[q]])
          if (c != E) cand.push_back(c);
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      std::vector<int32_t> out{E};
      for (int32_t c : cand) {
        bool all = true;
        for (const V3 &p : pts) all = all && in_cell(c, p);
        if (all) out.push_back(c);
      }
      return out;
    };
    // the mean over cells of their projection's functional (mvals_of gives
    // the monomial values of the functional in cell c's basis)
    auto mean_cell_rows = [&](const std::vector<int32_t> &cells, const std::function<void(int32_t, double *)> &mvals_of,
                              Row &R) {
      const int Nk = vem::npoly3(k);
      const double wgt = 1.0 / static_cast<double>(cells.size());
      for (int32_t c : cells) {
        double mv[10];
        mvals_of(c, mv);
        const std::vector<int32_t> craw = cell_raw_dofs(Mc, c);
        const int nE = static_cast<int>(craw.size());
        for (int r = 0; r < nE; ++r) {
          double sum = 0;
          for (int a = 0; a < Nk; ++a) sum += mv[a] * cproj[c].Pis[a * nE + r];
          if (sum != 0.0) R.e.push_back({craw[r], wgt * sum});
        }
      }
    };
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < Mf.nc(); ++c) {
      const int32_t E = par[c];
      const vem::Cell &cc = ccell[E];
      const vem::CellData &pj = cproj[E];
      const std::vector<int32_t> craw = cell_raw_dofs(Mc, E);
      const int Nk = vem::npoly3(k), Nf2 = vem::npoly2(k);
      const int nE = static_cast<int>(craw.size());
      auto cell_row = [&](const double *mvals, Row &R) {
        for (int r = 0; r < nE; ++r) {
          double s = 0;
          for (int a = 0; a < Nk; ++a) s += mvals[a] * pj.Pis[a * nE + r];
          if (s != 0.0) R.e.push_back({craw[r], s});
        }
      };
      auto face_row = [&](int64_t f, const double *mvals, Row &R) {
        const std::vector<int32_t> fr = face_raw(f);
        const vem::FaceProj &fp = fproj[f];
        for (int r = 0; r < fp.nd; ++r) {
          double s = 0;
          for (int a = 0; a < Nf2; ++a) s += mvals[a] * fp.Pi[a * fp.nd + r];
          if (s != 0.0) R.e.push_back({fr[r], s});
        }
      };
      auto in_face = [&](int64_t f, V3 p) {
        const std::vector<V3> P = face_points(Mc, static_cast<int32_t>(f), 1);
        const V3 n = Mc.fnormal[f];
        if (std::fabs(dot(n, p - P[0])) > tol) return false;
        for (size_t i = 0; i < P.size(); ++i) {
          const V3 on = cross(P[(i + 1) % P.size()] - P[i], n);
          if (dot(on, p - P[i]) > tol * norm(on)) return false;
        }
        return true;
      };
      // a point sits on a coarse vertex or edge within the weld distance:
      // such points are there up to rounding, and a looser test can take a
      // point next to a tiny feature for one on a neighbouring edge
      auto point_row = [&](V3 p, Row &R) {
        for (int64_t q = Mc.cvptr[E]; q < Mc.cvptr[E + 1]; ++q)
          if (norm(Mc.X[Mc.cvert[q]] - p) < kVertTol) {
            R.e.push_back({Mc.cvert[q], 1.0});
            return;
          }
        for (int64_t q = Mc.ceptr[E]; q < Mc.ceptr[E + 1]; ++q) {
          const int32_t e = Mc.cedge[q];
          const V3 a = Mc.X[Mc.edges[e][0]], b = Mc.X[Mc.edges[e][1]], ab = b - a;
          const double tau = dot(p - a, ab) / dot(ab, ab);
          if (tau > 0 && tau < 1 && norm(p - a - tau * ab) < kVertTol) {
            if (k == 1) {
              R.e.push_back({Mc.edges[e][0], 1 - tau});
              R.e.push_back({Mc.edges[e][1], tau});
            } else {
              R.e.push_back({Mc.edges[e][0], 2 * (tau - 0.5) * (tau - 1)});
              R.e.push_back({static_cast<int32_t>(Mc.nv() + e), -4 * tau * (tau - 1)});
              R.e.push_back({Mc.edges[e][1], 2 * tau * (tau - 0.5)});
            }
            return;
          }
        }
        for (int64_t q = Mc.cfptr[E]; q < Mc.cfptr[E + 1]; ++q) {
          const int32_t f = Mc.cface[q];
          if (in_face(f, p)) {
            double mv[6];
            fproj[f].eval(p, k, mv);
            face_row(f, mv, R);
            return;
          }
        }
        double mv[10];
        pj.basis.eval(p, k, mv);
        cell_row(mv, R);
      };
      // naive prolongation of a point: shared vertex or edge-midpoint DOFs
      // copy, any other point takes the mean of the projections of the
      // coarse cells holding it
      auto naive_point_row = [&](V3 p, Row &R) {
        for (int64_t q = Mc.cvptr[E]; q < Mc.cvptr[E + 1]; ++q)
          if (norm(Mc.X[Mc.cvert[q]] - p) < kVertTol) {
            R.e.push_back({Mc.cvert[q], 1.0});
            return;
          }
        if (k == 2)
          for (int64_t q = Mc.ceptr[E]; q < Mc.ceptr[E + 1]; ++q) {
            const int32_t e = Mc.cedge[q];
            if (norm(0.5 * (Mc.X[Mc.edges[e][0]] + Mc.X[Mc.edges[e][1]]) - p) < kVertTol) {
              R.e.push_back({static_cast<int32_t>(Mc.nv() + e), 1.0});
              return;
            }
          }
        mean_cell_rows(cells_holding(E, {p}), [&](int32_t cc2, double *mv) { cproj[cc2].basis.eval(p, k, mv); }, R);
      };
      const std::vector<int32_t> fraw = cell_raw_dofs(Mf, c);
      for (int32_t r : fraw) {
        if (owner[r] != c) continue;
        Row &R = rows[r];
        const int kind = raw_kind(Mf, r);
        if (kind <= 1) {
          if (naive) naive_point_row(raw_point(Mf, r), R);
          else point_row(raw_point(Mf, r), R);
        } else if (kind == 2) {
          const int64_t f = r - Mf.nv() - Mf.ne();
          const std::vector<V3> P = face_points(Mf, static_cast<int32_t>(f), 1);
          // area centroid and area of the fine face
          const V3 av = geo::area_vector(P);
          const double ar = norm(av);
          V3 cen;
          double A2 = 0;
          for (size_t i = 1; i + 1 < P.size(); ++i) {
            const double t = dot(cross(P[i] - P[0], P[i + 1] - P[0]), (1.0 / ar) * av);
            A2 += t;
            cen = cen + t * (P[0] + P[i] + P[i + 1]);
          }
          cen = (1.0 / (3.0 * A2)) * cen;
          // the fine face lies in the coarse face's plane when all of its
          // vertices do (a distance test: the computed normal of a sliver
          // face can be off by far more than its vertices are)
          std::vector<int32_t> coplanar;
          for (int64_t q = Mc.cfptr[E]; q < Mc.cfptr[E + 1]; ++q) {
            const int32_t F2 = Mc.cface[q];
            const V3 o = Mc.X[Mc.fvert[Mc.fptr[F2]]];
            bool planar = true;
            for (const V3 &p : P) planar = planar && std::fabs(dot(Mc.fnormal[F2], p - o)) <= tol;
            if (planar) coplanar.push_back(F2);
          }
          bool done = false;
          // a coarse face equal to the fine face is its host before any face
          // the fine centroid is merely near (a tiny fine face beside a coarse
          // edge passes the containment slack of the neighbouring face)
          for (int32_t F2 : coplanar) {
            const vem::FaceProj &fp = fproj[F2];
            if (std::fabs(fp.area - ar) < 1e-12 * ar && norm(fp.xf - cen) < tol) {
              R.e.push_back({static_cast<int32_t>(Mc.nv() + Mc.ne() + F2), 1.0});
              done = true;
              break;
            }
          }
          if (naive && !done) {
            // the mean over the coarse cells holding the fine face of their
            // projection's mean on it
            mean_cell_rows(cells_holding(E, P), [&](int32_t cc2, double *mv) { vem::polygon_mean(P, cproj[cc2].basis, k, mv); }, R);
            done = true;
          }
          for (size_t t = 0; t < coplanar.size() && !done; ++t) {
            const int32_t F2 = coplanar[t];
            if (!in_face(F2, cen)) continue;
            double mv[6];
            vem::polygon_mean_face(P, fproj[F2], k, mv);
            face_row(F2, mv, R);
            done = true;
          }
          if (!done) {
            double mv[10];
            vem::polygon_mean(P, pj.basis, k, mv);
            cell_row(mv, R);
          }
        } else {
          const double vf = Mf.cvol[c];
          if (std::fabs(vf - Mc.cvol[E]) < 1e-12 * vf && norm(Mf.ccen[c] - Mc.ccen[E]) < tol) {
            R.e.push_back({static_cast<int32_t>(Mc.nv() + Mc.ne() + Mc.nf() + E), 1.0});
          } else {
            std::vector<std::vector<V3>> fpts;
            for (int64_t q = Mf.cfptr[c]; q < Mf.cfptr[c + 1]; ++q) fpts.push_back(face_points(Mf, Mf.cface[q], Mf.corient[q]));
            double mv[10];
            vem::polyhedron_mean(fpts, pj.basis, k, mv);
            cell_row(mv, R);
          }
        }
      }
    }
    // CSR in ordered free numbering
    std::vector<int32_t> frow(F.nfree, -1);   // free fine -> raw
    for (int64_t r = 0; r < nrf; ++r) {
      const int32_t fi = F.free[F.perm[r]];
      if (fi >= 0) frow[fi] = static_cast<int32_t>(r);
    }
    rp.assign(F.nfree + 1, 0);
    // each row is finished on its own (in parallel, in place), then the
    // rows are concatenated in order
#pragma omp parallel
    {
      std::vector<std::pair<int32_t, double>> ent;   // per-thread scratch
#pragma omp for schedule(dynamic, 4096)
      for (int64_t i = 0; i < F.nfree; ++i) {
        auto &E = rows[frow[i]].e;
        // weights at rounding level of the row's largest weight are zeros of
        // the exact prolongation; dropped so that no coarse DOF keeps a
        // numerically empty column
        double wmax = 0;
        for (auto &e : E) wmax = std::max(wmax, std::fabs(e.second));
        ent.clear();
        for (auto &e : E) {
          const int32_t cj = C.free[C.perm[e.first]];
          if (cj >= 0 && std::fabs(e.second) > 1e-13 * wmax) ent.push_back({cj, e.second});
        }
        std::sort(ent.begin(), ent.end());
        // merge duplicates (a coarse DOF reached twice), written back over
        // the row (never longer than it was)
        size_t m = 0;
        for (auto &e : ent) {
          if (m > 0 && E[m - 1].first == e.first) E[m - 1].second += e.second;
          else E[m++] = e;
        }
        E.resize(m);
        rp[i + 1] = static_cast<int64_t>(m);
      }
    }
    for (int64_t i = 0; i < F.nfree; ++i) rp[i + 1] += rp[i];
    ci.resize(rp[F.nfree]);
    va.resize(rp[F.nfree]);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < F.nfree; ++i) {
      auto &E = rows[frow[i]].e;
      int64_t q = rp[i];
      for (auto &e : E) {
        ci[q] = e.first;
        va[q] = e.second;
        ++q;
      }
      std::vector<std::pair<int32_t, double>>().swap(E);   // freed here, in parallel
    }
  }
  std::unordered_map<uint64_t, int32_t> cedge_map;

  // ------------------------------------------------------------------ driver
  void run() {
    build_forest();
    progress("grid: %zu cut-cell trees", trees.size());
    levels.push_back(initial_level());
    make_tiles(levels[0]);
    conform(levels[0]);
    number_dofs(levels[0]);
    progress("grid: level 0 has %lld cells and %lld DOFs", static_cast<long long>(levels[0].mesh.nc()),
             static_cast<long long>(levels[0].nfree));
    int t = 0;
    while (true) {
      const int64_t n_here = levels.back().nfree;
      if (t >= L - 1 && n_here <= coarse_max) break;
      if (static_cast<int>(levels.size()) >= max_levels) break;
      bool changed = false;
      Level nl = coarsen(levels.back(), &changed);
      if (!changed) break;
      make_tiles(nl);
      conform(nl);
      number_dofs(nl);
      // parent map
      const Level &f = levels.back();
      std::vector<int32_t> tile_cell(nl.tiles.size(), -1);
      for (int64_t c = 0; c < nl.mesh.nc(); ++c) tile_cell[nl.mesh.ctile[c]] = static_cast<int32_t>(c);
      std::vector<int32_t> par(f.mesh.nc());
      for (int64_t c = 0; c < f.mesh.nc(); ++c) {
        const Tile &T = f.tiles[f.mesh.ctile[c]];
        int32_t ct = -1;
        int64_t corner;
        if (T.type == 0 && nl.E[trees[T.tree].bg] < 0) {
          int a = T.node;
          std::vector<int> path;
          while (a >= 0) {
            path.push_back(a);
            a = trees[T.tree].nodes[a].parent;
          }
          for (auto it = path.rbegin(); it != path.rend(); ++it)
            if (!nl.act[T.tree][*it]) {
              for (int32_t q : nl.tree_tiles[T.tree])
                if (nl.tiles[q].node == *it) ct = q;
              break;
            }
        } else {
          corner = T.type == 0 ? trees[T.tree].bg : bgi(N, T.lo[0], T.lo[1], T.lo[2]);
          ct = nl.cube_tile[corner];
        }
        if (ct < 0 || tile_cell[ct] < 0) throw std::runtime_error("hierarchy is not nested");
        par[c] = tile_cell[ct];
      }
      parents.push_back(std::move(par));
      levels.push_back(std::move(nl));
      // prolongation into the fine level, dropping unused coarse DOFs
      std::vector<int64_t> rp;
      std::vector<int32_t> ci;
      std::vector<double> va;
      prolongation(static_cast<int>(levels.size()) - 2, rp, ci, va);
      // a coarse DOF is used when some fine DOF depends on it with a weight
      // above 1e-10; smaller largest weights are exact zeros of the
      // projection polluted by rounding (thin cells amplify it)
      std::vector<uint8_t> used(levels.back().nfree, 0);
      {
        std::vector<double> cmax(levels.back().nfree, 0.0);
        for (size_t q = 0; q < ci.size(); ++q) cmax[ci[q]] = std::max(cmax[ci[q]], std::fabs(va[q]));
        for (int64_t j = 0; j < levels.back().nfree; ++j) used[j] = cmax[j] > 1e-10;
      }
      bool all = true;
      for (uint8_t u : used) all = all && u;
      if (!all) {
        // entries of unused columns are removed with the columns (rows
        // counted, then filled, in parallel)
        const int64_t nr = static_cast<int64_t>(rp.size()) - 1;
        std::vector<int64_t> rp2(rp.size(), 0);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nr; ++i) {
          int64_t c = 0;
          for (int64_t q = rp[i]; q < rp[i + 1]; ++q) c += used[ci[q]];
          rp2[i + 1] = c;
        }
        for (int64_t i = 0; i < nr; ++i) rp2[i + 1] += rp2[i];
        std::vector<int32_t> remap(levels.back().nfree, -1);
        int32_t q = 0;
        for (int64_t j = 0; j < levels.back().nfree; ++j)
          if (used[j]) remap[j] = q++;
        std::vector<int32_t> ci2(rp2[nr]);
        std::vector<double> va2(rp2[nr]);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nr; ++i) {
          int64_t o = rp2[i];
          for (int64_t r = rp[i]; r < rp[i + 1]; ++r)
            if (used[ci[r]]) {
              ci2[o] = remap[ci[r]];
              va2[o] = va[r];
              ++o;
            }
        }
        rp.swap(rp2);
        ci.swap(ci2);
        va.swap(va2);
        drop_unused(levels.back(), used);
      }
      progress("grid: level %zu has %lld cells and %lld DOFs", levels.size() - 1,
               static_cast<long long>(levels.back().mesh.nc()), static_cast<long long>(levels.back().nfree));
      out->P.push_back({std::move(rp), std::move(ci), std::move(va)});
      ++t;
    }
    emit();
    progress("grid: element operators done");
  }

  void emit() {
    Output &o = *out;
    const int nl = static_cast<int>(levels.size());
    o.levels.resize(nl);
    for (int l = 0; l < nl; ++l) {
      const Level &lv = levels[l];
      const Mesh &M = lv.mesh;
      LevelOut &L = o.levels[l];
      L.n_dof = lv.nfree;
      L.cell_ptr.assign(1, 0);
      L.cell_dof.clear();
      for (int64_t c = 0; c < M.nc(); ++c) {
        for (int32_t r : cell_raw_dofs(M, c)) L.cell_dof.push_back(lv.free[lv.perm[r]]);
        L.cell_ptr.push_back(static_cast<int64_t>(L.cell_dof.size()));
      }
      if (l + 1 < nl) L.parent = parents[l];
      L.n_cells = M.nc();
      L.dof_point.assign(3 * lv.nfree, 0.0);
      L.dof_kind.assign(lv.nfree, 0);
      for (int64_t r = 0; r < raw_count(M); ++r) {
        const int32_t fi = lv.free[lv.perm[r]];
        if (fi < 0) continue;
        const V3 p = raw_point(M, r);
        L.dof_point[3 * fi] = p.x;
        L.dof_point[3 * fi + 1] = p.y;
        L.dof_point[3 * fi + 2] = p.z;
        L.dof_kind[fi] = static_cast<int8_t>(raw_kind(M, r));
      }
    }
    // finest-level element operators; uncut cubes share one block per shape
    const Level &l0 = levels[0];
    const Mesh &M = l0.mesh;
    const int64_t nc = M.nc();
    o.n_vert = M.nv();
    o.X = M.X;
    o.cell_vptr.assign(nc + 1, 0);
    for (int64_t c = 0; c < nc; ++c) o.cell_vptr[c + 1] = o.cell_vptr[c] + (M.cvptr[c + 1] - M.cvptr[c]);
    o.cell_vert.assign(M.cvert.begin(), M.cvert.end());
    o.ke_off.assign(nc, 0);
    o.be_off.assign(nc, 0);
    o.vc_off.assign(nc, 0);
    std::vector<vem::CellData> data(nc);
    std::vector<int64_t> tmpl(nc, -1);
    std::unordered_map<int, int64_t> shape;   // plain cube side -> first cell
    for (int64_t c = 0; c < nc; ++c)
      if (M.cplain[c]) {
        auto it = shape.find(M.cside[c]);
        if (it == shape.end()) shape[M.cside[c]] = c;
        else tmpl[c] = it->second;
      }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < nc; ++c)
      if (tmpl[c] < 0) data[c] = vem::element(vem_cell(M, c), k, true);
    // a degenerate cell (e.g. a sliver edge far below the grid spacing) must
    // not pass unnoticed into the operators
    for (int64_t c = 0; c < nc; ++c) {
      if (tmpl[c] >= 0) continue;
      bool ok = true;
      for (double v : data[c].K) ok = ok && std::isfinite(v);
      for (double v : data[c].B) ok = ok && std::isfinite(v);
      for (double v : data[c].V) ok = ok && std::isfinite(v);
      if (ok) continue;
      if (const char *dump = std::getenv("FVEM_DUMP_CELL")) {
        // outward faces as vertex cycles, for offline inspection
        const vem::Cell C = vem_cell(M, c);
        if (FILE *fp = std::fopen(dump, "w")) {
          std::fprintf(fp, "%zu %zu\n", C.X.size(), C.faces.size());
          for (const V3 &x : C.X) std::fprintf(fp, "%.17g %.17g %.17g\n", x.x, x.y, x.z);
          for (const auto &f : C.faces) {
            std::fprintf(fp, "%zu", f.size());
            for (int q : f) std::fprintf(fp, " %d", q);
            std::fprintf(fp, "\n");
          }
          std::fclose(fp);
        }
      }
      throw std::runtime_error("the VEM operators of cell " + std::to_string(c) + " are not finite");
    }
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t src = tmpl[c] < 0 ? c : tmpl[c];
      if (src == c) {
        o.ke_off[c] = static_cast<int64_t>(o.ke_val.size());
        o.ke_val.insert(o.ke_val.end(), data[c].K.begin(), data[c].K.end());
        o.be_off[c] = static_cast<int64_t>(o.be_val.size());
        o.be_val.insert(o.be_val.end(), data[c].B.begin(), data[c].B.end());
        o.vc_off[c] = static_cast<int64_t>(o.vc_val.size());
        o.vc_val.insert(o.vc_val.end(), data[c].V.begin(), data[c].V.end());
      } else {
        o.ke_off[c] = o.ke_off[src];
        o.be_off[c] = o.be_off[src];
        o.vc_off[c] = o.vc_off[src];
      }
    }
    // cell geometry for the velocity operators: centroid, diameter, volume
    o.cell_geom.assign(5 * nc, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
      double hE = 0;
      for (int64_t a = M.cvptr[c]; a < M.cvptr[c + 1]; ++a)
        for (int64_t b = a + 1; b < M.cvptr[c + 1]; ++b) hE = std::max(hE, norm(M.X[M.cvert[a]] - M.X[M.cvert[b]]));
      const V3 xc = tmpl[c] < 0 ? data[c].basis.xc : M.ccen[c];
      o.cell_geom[5 * c] = xc.x;
      o.cell_geom[5 * c + 1] = xc.y;
      o.cell_geom[5 * c + 2] = xc.z;
      o.cell_geom[5 * c + 3] = hE;
      o.cell_geom[5 * c + 4] = M.cvol[c];
    }
    o.n_shared_blocks = static_cast<int64_t>(shape.size());
    // pure-Neumann components: connected cells (sharing DOFs) without an eliminated DOF
    const LevelOut &L0 = o.levels[0];
    std::vector<int64_t> parent(L0.n_dof);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int64_t x) {
      while (parent[x] != x) x = parent[x] = parent[parent[x]];
      return x;
    };
    std::vector<uint8_t> cell_anchored(nc, 0);
    for (int64_t c = 0; c < nc; ++c) {
      int64_t first = -1;
      for (int64_t q = L0.cell_ptr[c]; q < L0.cell_ptr[c + 1]; ++q) {
        const int32_t d = L0.cell_dof[q];
        if (d < 0) {
          cell_anchored[c] = 1;
          continue;
        }
        if (first < 0) first = d;
        else {
          const int64_t a = find(first), b = find(d);
          if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
      }
    }
    std::vector<uint8_t> anchored(L0.n_dof, 0);
    for (int64_t c = 0; c < nc; ++c)
      if (cell_anchored[c])
        for (int64_t q = L0.cell_ptr[c]; q < L0.cell_ptr[c + 1]; ++q)
          if (L0.cell_dof[q] >= 0) anchored[find(L0.cell_dof[q])] = 1;
    o.component.assign(L0.n_dof, -1);
    std::unordered_map<int64_t, int32_t> cid;
    for (int64_t i = 0; i < L0.n_dof; ++i) {
      const int64_t r = find(i);
      if (anchored[r]) continue;
      auto it = cid.find(r);
      if (it == cid.end()) it = cid.emplace(r, static_cast<int32_t>(cid.size())).first;
      o.component[i] = it->second;
    }
    o.n_components = static_cast<int32_t>(cid.size());
    // DOF support points of the finest level (ordered free numbering)
    o.dof_point.assign(3 * L0.n_dof, 0.0);
    o.dof_kind.assign(L0.n_dof, 0);
    for (int64_t r = 0; r < raw_count(M); ++r) {
      const int32_t fi = l0.free[l0.perm[r]];
      if (fi < 0) continue;
      const V3 p = raw_point(M, r);
      o.dof_point[3 * fi] = p.x;
      o.dof_point[3 * fi + 1] = p.y;
      o.dof_point[3 * fi + 2] = p.z;
      o.dof_kind[fi] = static_cast<int8_t>(raw_kind(M, r));
    }
    o.n_trees = static_cast<int64_t>(trees.size());
    export_locator(o);
    // outward face cycles of the finest cells
    o.cell_face_ptr.assign(1, 0);
    o.face_ptr.assign(1, 0);
    o.face_vert.clear();
    for (int64_t c = 0; c < M.nc(); ++c) {
      for (int64_t q = M.cfptr[c]; q < M.cfptr[c + 1]; ++q) {
        const int32_t f = M.cface[q];
        const size_t at = o.face_vert.size();
        o.face_vert.insert(o.face_vert.end(), M.fvert.begin() + M.fptr[f], M.fvert.begin() + M.fptr[f + 1]);
        if (M.corient[q] < 0) std::reverse(o.face_vert.begin() + at, o.face_vert.end());
        o.face_ptr.push_back(static_cast<int64_t>(o.face_vert.size()));
      }
      o.cell_face_ptr.push_back(static_cast<int64_t>(o.face_ptr.size()) - 1);
    }
  }

  // point location and triangle lists of the finest level (see Output)
  void export_locator(Output &o) const {
    const Level &l0 = levels[0];
    const Mesh &M = l0.mesh;
    const int64_t N3 = static_cast<int64_t>(N) * N * N;
    o.loc_bg.assign(N3, -1);
    o.loc_tree_root.resize(trees.size());
    int64_t nn = 0;
    for (size_t t = 0; t < trees.size(); ++t) {
      o.loc_tree_root[t] = static_cast<int32_t>(nn);
      nn += static_cast<int64_t>(trees[t].nodes.size());
    }
    if (nn >= (int64_t(1) << 31)) throw std::runtime_error("too many BSP nodes for int32 indices");
    o.loc_plane.assign(4 * nn, 0.0);
    o.loc_child.assign(2 * nn, -1);
    o.loc_cell.assign(nn, -1);
    for (size_t t = 0; t < trees.size(); ++t) {
      const int32_t r = o.loc_tree_root[t];
      o.loc_bg[trees[t].bg] = -2 - static_cast<int32_t>(t);
      for (size_t a = 0; a < trees[t].nodes.size(); ++a) {
        const Node &nd = trees[t].nodes[a];
        if (nd.child[0] < 0) continue;
        const int64_t gq = r + static_cast<int64_t>(a);
        o.loc_plane[4 * gq] = nd.n.x;
        o.loc_plane[4 * gq + 1] = nd.n.y;
        o.loc_plane[4 * gq + 2] = nd.n.z;
        o.loc_plane[4 * gq + 3] = nd.d;
        o.loc_child[2 * gq] = r + nd.child[0];
        o.loc_child[2 * gq + 1] = r + nd.child[1];
      }
    }
    for (int64_t c = 0; c < M.nc(); ++c) {
      const Tile &T = l0.tiles[M.ctile[c]];
      if (T.type == 1) {
        if (T.hi[0] - T.lo[0] != 1) throw std::runtime_error("finest-level cube larger than one background cell");
        o.loc_bg[bgi(N, T.lo[0], T.lo[1], T.lo[2])] = static_cast<int32_t>(c);
      } else {
        o.loc_cell[o.loc_tree_root[T.tree] + T.node] = static_cast<int32_t>(c);
      }
    }
    o.tri_ptr.assign(N3 + 1, 0);
    for (size_t q = 0; q < tri_cells.size(); ++q) o.tri_ptr[tri_cells[q] + 1] = static_cast<int64_t>(tri_lists[q].size());
    for (int64_t b = 0; b < N3; ++b) o.tri_ptr[b + 1] += o.tri_ptr[b];
    o.tri_id.resize(o.tri_ptr[N3]);
    for (size_t q = 0; q < tri_cells.size(); ++q)
      std::copy(tri_lists[q].begin(), tri_lists[q].end(), o.tri_id.begin() + o.tri_ptr[tri_cells[q]]);
    o.tri_xyz.resize(9 * TF.size());
    for (size_t t = 0; t < TF.size(); ++t)
      for (int c = 0; c < 3; ++c) {
        o.tri_xyz[9 * t + 3 * c] = TV[TF[t][c]].x;
        o.tri_xyz[9 * t + 3 * c + 1] = TV[TF[t][c]].y;
        o.tri_xyz[9 * t + 3 * c + 2] = TV[TF[t][c]].z;
      }
  }
};

void build_grid(const Input &in, Output *out) {
  BuilderImpl b;
  b.N = in.N;
  b.k = in.k;
  b.L = in.L;
  b.h = 1.0 / in.N;
  b.dirichlet = in.dirichlet;
  b.coarse_max = in.coarse_max;
  b.max_levels = in.max_levels;
  b.naive = in.naive;
  b.out = out;
  b.TV.resize(in.nv);
  for (int64_t i = 0; i < in.nv; ++i) b.TV[i] = V3(in.V[3 * i], in.V[3 * i + 1], in.V[3 * i + 2]);
  b.TF.resize(in.nt);
  b.tn.resize(in.nt);
  b.td.resize(in.nt);
  b.tarea.resize(in.nt);
  for (int64_t t = 0; t < in.nt; ++t) {
    for (int d = 0; d < 3; ++d) b.TF[t][d] = in.F[3 * t + d];
    const V3 a = b.TV[b.TF[t][0]], c1 = b.TV[b.TF[t][1]], c2 = b.TV[b.TF[t][2]];
    const V3 n = cross(c1 - a, c2 - a);
    const double l = norm(n);
    b.tn[t] = (1.0 / l) * n;
    b.td[t] = dot(b.tn[t], a);
    b.tarea[t] = 0.5 * l;
    b.total_area += 0.5 * l;
  }
  b.run();
}

}  // namespace fvem::grid
