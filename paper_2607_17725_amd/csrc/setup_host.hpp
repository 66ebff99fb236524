// Host-side setup of the multigrid hierarchy: validation, assembly of CSR
// operators from element blocks, the element-wise Galerkin product and CSR
// transposes.  Pure C++17 (OpenMP); no HIP calls.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fvem.h"

namespace fvem {

struct HostCSR {
  int64_t n_rows = 0, n_cols = 0;
  std::vector<int64_t> rp;   // n_rows + 1
  std::vector<int32_t> ci;
  std::vector<double> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Cells of one level: local DOF lists (free index or -1).
struct HostCells {
  int64_t n_cells = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> dof;
};

// Dense element blocks, block c is n_c x m_c row-major at off[c] (blocks
// may be shared between cells of identical shape).
struct HostBlocks {
  std::vector<int64_t> off;
  std::vector<double> val;
};

struct SetupError {
  fvem_status code;
  std::string msg;
};

// Assemble y = sum_c scatter(block_c) into a CSR with rows/cols given by
// the row DOF lists (rows) and column lists (cols) of each cell.  Entries
// with a negative index are skipped.  Deterministic: contributions to an
// entry are summed in increasing cell order.
HostCSR assemble_blocks(int64_t n_rows, int64_t n_cols, const HostCells &rows, const HostCells &cols,
                        const HostBlocks &blocks);

// Element-wise Galerkin product: for each coarse cell E,
//   K_E = sum_{fine cells f with parent[f] = E} P_f^T K_f P_f
// where P_f is the dense block of P's rows of f's DOFs restricted to E's
// DOFs.  Throws SetupError(INVALID) if a row references a DOF outside E.
HostBlocks galerkin_blocks(const HostCells &fine, const HostBlocks &kf, const int32_t *parent,
                           const HostCells &coarse, const HostCSR &P);

HostCSR transpose(const HostCSR &A);

// Level order of the sliced storage: inside each window of w consecutive
// rows, rows by decreasing length (stable).  Returns order[new] = old.
std::vector<int32_t> window_order(const HostCSR &A, int64_t w);

// B = rows order[r] of A with columns renamed by col_map (old -> new; null
// keeps them), columns sorted ascending within each row.
HostCSR permute(const HostCSR &A, const std::vector<int32_t> &order, const std::vector<int32_t> *col_map);

// Sliced ELLPACK (64-row slices, column-major inside a slice); padding has
// value 0 and column min(row, n_cols - 1).
struct HostSELL {
  int64_t n = 0, m = 0, nnz = 0, nslices = 0;
  std::vector<int64_t> sp;   // nslices + 1, in entries
  std::vector<int32_t> sl;   // longest row per slice
  std::vector<int32_t> rl;   // row lengths
  std::vector<int32_t> ci;
  std::vector<double> v;
};
HostSELL to_sell(const HostCSR &A);
HostCSR from_sell(const HostSELL &S);

// max_i sum_j |a_ij| / sqrt(a_ii a_jj): Gershgorin bound of D^-1/2 A D^-1/2,
// which has the spectrum of D^-1 A and stays bounded by the row length for
// symmetric positive semi-definite A even where some a_ii are tiny.
double gershgorin_scaled(const HostCSR &A);

// Floating components of a symmetric matrix graph: connected components whose
// rows sum to ~0 (pure-Neumann constants).  Returns per-row id or -1.
std::vector<int32_t> floating_components(const HostCSR &A, int32_t *n_comp);

}  // namespace fvem
