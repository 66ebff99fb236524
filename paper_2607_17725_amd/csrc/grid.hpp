// Native grid builder interface (implemented in grid.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "geom.hpp"
#include "vem.hpp"

namespace fvem::grid {

struct Input {
  const double *V = nullptr;   // boundary mesh vertices [nv x 3]
  int64_t nv = 0;
  const int32_t *F = nullptr;  // outward triangles [nt x 3]
  int64_t nt = 0;
  int N = 16;                  // background grid N^3 on the unit cube
  int k = 1;                   // VEM order of the pressure
  int L = 5;                   // hierarchy levels (paper: 5)
  bool dirichlet = false;      // p = 0 on z = 1
  int64_t coarse_max = 16384;  // keep coarsening while the coarsest level is larger
  int max_levels = 12;
  bool naive = false;          // the naive prolongation of Sec. 4 (ablation) instead of the diffusion-free one
};

struct LevelOut {
  int64_t n_dof = 0, n_cells = 0;
  std::vector<double> dof_point;   // [n_dof x 3] support points (ordered free numbering)
  std::vector<int8_t> dof_kind;    // 0 vertex, 1 edge midpoint, 2 face, 3 cell
  std::vector<int64_t> cell_ptr;
  std::vector<int32_t> cell_dof;
  std::vector<int32_t> parent;
};

struct CSROut {
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

struct Output {
  std::vector<LevelOut> levels;
  std::vector<CSROut> P;        // P[l]: level l+1 -> level l
  std::vector<int64_t> ke_off, be_off, vc_off;
  std::vector<double> ke_val, be_val, vc_val;
  std::vector<double> cell_geom;  // [n_cells x 5] centroid, h_E, volume
  int64_t n_vert = 0;
  std::vector<geo::V3> X;       // velocity vertices
  std::vector<int64_t> cell_vptr;
  std::vector<int32_t> cell_vert;
  std::vector<int32_t> component;
  int32_t n_components = 0;
  std::vector<double> dof_point;  // finest-level DOF support points [n_dof x 3]
  std::vector<int8_t> dof_kind;   // 0 vertex, 1 edge, 2 face, 3 cell
  int64_t n_shared_blocks = 0;
  int64_t n_trees = 0;
  // point location on the finest level: per background cell (index
  // (i N + j) N + k) the level-0 cube cell it is, -1 (no fluid cell), or
  // -2 - t for BSP tree t; tree t's nodes start at tree_root[t]; an inner
  // node splits by plane n.x = d (node_plane: n, d) into child[0] (n.x < d)
  // and child[1]; a leaf holds its level-0 cell or -1 (solid)
  std::vector<int32_t> loc_bg;
  std::vector<int32_t> loc_tree_root;
  std::vector<double> loc_plane;    // 4 per node
  std::vector<int32_t> loc_child;   // 2 per node, -1 at leaves
  std::vector<int32_t> loc_cell;    // per node: the leaf's cell or -1
  // boundary triangles overlapping each background cell (CSR over N^3)
  std::vector<int64_t> tri_ptr;
  std::vector<int32_t> tri_id;
  std::vector<double> tri_xyz;     // 9 per boundary triangle: its corners
  // faces of each finest-level cell as outward vertex cycles (velocity
  // vertex ids): cell c's faces are cell_face_ptr[c] .. cell_face_ptr[c+1]),
  // face f's corners face_vert[face_ptr[f] .. face_ptr[f+1])
  std::vector<int64_t> cell_face_ptr, face_ptr;
  std::vector<int32_t> face_vert;
};

void build_grid(const Input &in, Output *out);

}  // namespace fvem::grid
