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
// with a negative index are skipped.  Deterministic and translation
// invariant: contributions to an entry are summed in increasing order of
// value, so equal sets of contributions give bitwise equal entries.
HostCSR assemble_blocks(int64_t n_rows, int64_t n_cols, const HostCells &rows, const HostCells &cols,
                        const HostBlocks &blocks);

// Element-wise Galerkin product: for each coarse cell E,
//   K_E = sum_{fine cells f with parent[f] = E} P_f^T K_f P_f
// where P_f is the dense block of P's rows of f's DOFs restricted to E's
// DOFs.  Throws SetupError(INVALID) if a row references a DOF outside E.
HostBlocks galerkin_blocks(const HostCells &fine, const HostBlocks &kf, const int32_t *parent,
                           const HostCells &coarse, const HostCSR &P);

HostCSR transpose(const HostCSR &A);

// C = X Y (sparse products, columns sorted; each entry sums its terms in
// the order of X's row and then Y's rows, so the result is deterministic).
HostCSR multiply(const HostCSR &X, const HostCSR &Y);

// Galerkin operator A_c = P^T A P by sparse products, for prolongations
// whose rows may reach beyond one coarse cell (no element-wise form).
HostCSR galerkin_product(const HostCSR &A, const HostCSR &P);

// Level order of the sliced storage: inside each window of w consecutive
// rows (w a multiple of 64), rows by decreasing length (stable); then the
// window's full 64-row chunks ordered by their smallest original row, so the
// slices of one part of the grid are adjacent.  Returns order[new] = old.
std::vector<int32_t> window_order(const HostCSR &A, int64_t w);

// B = rows order[r] of A with columns renamed by col_map (old -> new; null
// keeps them), columns sorted ascending within each row.  order may be
// longer than A's row count and hold -1 (empty rows); n_cols < 0 keeps A's
// column count.
HostCSR permute(const HostCSR &A, const std::vector<int32_t> &order, const std::vector<int32_t> *col_map,
                int64_t n_cols = -1);

// Sliced ELLPACK with 64-row slices, interleaved in groups of 4 entries:
// entry j of row 64 s + r sits at sp[s] + 256 (j / 4) + 4 r + j % 4, so a
// wavefront reads each group of 4 entries of its 64 rows as one contiguous
// 1 KiB block (one 16-byte load per lane).  Slice widths are rounded up to a
// multiple of 4; padding has value 0 and column min(row, n_cols - 1).
//
// Value templates: away from cut cells a level operator repeats a few rows
// up to translation (one per DOF kind), so with each row's entries ordered
// by value the value sequences coincide.  Rows whose sequence is shared by
// at least min_uses rows read their values from a small template table; a
// slice whose rows all use templates stores no values.  Columns are stored
// for every row.  Two value sets share the columns: the FP64 values use
// templates only where rows are bitwise equal; the FP32 values (applied in
// single precision) also where rows agree to 1e-9 of their largest entry.
struct HostValues {
  std::vector<int64_t> vp;   // per slice: value offset, or -1 (all rows templated)
  std::vector<double> v;     // values of the explicit slices, same layout as ci
  std::vector<int32_t> tid;  // nslices * 64: template of each row (-1: explicit; 0 on padding rows)
  int32_t nt = 0, tw = 0;    // templates and their padded width (a multiple of 4)
  std::vector<double> tv;    // nt * tw template values
  int64_t nnz_explicit = 0, rows_templated = 0;
};
//
// Column codes: a slice whose columns fall in at most 64 aligned blocks of
// 1024 columns stores 16-bit codes (block index << 10 | offset in block) and
// a 64-entry table of block starts; other slices store int32 columns.
struct HostSELL {
  int64_t n = 0, m = 0, nnz = 0, nslices = 0;
  std::vector<int64_t> sp;   // nslices + 1, logical slice offsets (entries)
  std::vector<int32_t> sl;   // longest row per slice, rounded up to a multiple of 4
  std::vector<int32_t> rl;   // row lengths
  std::vector<int64_t> cp;   // per slice: offset of its columns in ci (bt < 0) or c16 (bt >= 0)
  std::vector<int64_t> bt;   // per slice: offset of its block table in btab, or -1
  std::vector<int32_t> ci;   // int32 columns of the slices without codes
  std::vector<uint16_t> c16; // column codes
  std::vector<int32_t> btab; // block starts, 64 per coded slice
  HostValues v64, v32;       // exact (FP64) and single-precision value sets
  int64_t at(int64_t s, int j, int r) const { return 256 * static_cast<int64_t>(j >> 2) + 4 * r + (j & 3); }
  int32_t col(int64_t s, int j, int r) const {
    const int64_t o = cp[s] + at(s, j, r);
    if (bt[s] < 0) return ci[o];
    return btab[bt[s] + (c16[o] >> 10)] + (c16[o] & 1023);
  }
};
// entries of every row ordered by (value, column) when templates are used;
// codes: 16-bit column codes where a slice's columns allow
HostSELL to_sell(const HostCSR &A, bool templates = false, int min_uses = 64, int max_templates = 1024,
                 bool codes = false);
HostCSR from_sell(const HostSELL &S);   // FP64 values

// Lattice stencil part of a level operator (compact storage of regular
// regions).  Away from cut cells every row of a DOF on the structured
// lattice (half-lattice of spacing h/2 for k = 2) is the same stencil up to
// translation, one stencil per parity class of the lattice coordinates.
// Such rows need no column or value storage: their columns follow from the
// lattice position, their values from one table per class.
//
// Level vectors are laid out by 8x8x8-point lattice tiles: every tile that
// holds a DOF gets 512 slots, class-major (8 classes of 4x4x4 points, the
// class of (a, b, c) being 4 (a & 1) + 2 (b & 1) + (c & 1)), so the slot of
// point (a, b, c) is tile_base[tile] + 64 class + 16 ((a & 7) >> 1) +
// 4 ((b & 7) >> 1) + ((c & 7) >> 1).  Slots without a DOF are holes (zero in
// every vector); DOFs off the lattice follow the slots.  A stencil kernel
// loads a tile's x plus a 2-point halo into LDS and applies the class
// tables; the other rows go to the sliced storage.
constexpr int STENCIL_MAX = 125;        // 5x5x5 offsets (|delta| <= 2 per axis)
constexpr int STENCIL_P2 = 8;           // LDS pitch of a halo row (6 points)
constexpr int STENCIL_P1 = 68;          // LDS pitch of a halo plane (6 rows)
constexpr int STENCIL_SUB = 6 * STENCIL_P1;   // LDS size of one class's 6^3 halo
struct HostLattice {
  int32_t lat_n = 0, tn = 0;         // lattice points and tiles per axis
  std::vector<int32_t> order;        // padded level order: order[slot] = DOF or -1
  std::vector<int32_t> tile_base;    // tn^3: first slot of each tile or -1
  std::vector<int32_t> tiles;        // tiles holding stencil rows (launch order)
  std::vector<uint64_t> mask;        // 8 words per entry of tiles: stencil slots
  std::vector<uint8_t> is_stencil;   // per DOF (caller order)
  int32_t len[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<int32_t> off;          // 8 x 128: LDS offset of each stencil entry
  std::vector<int32_t> delta;        // 8 x 128: lattice offset code (da+2)*25+(db+2)*5+(dc+2)
  std::vector<double> val;           // 8 x 128: entry values
  int64_t n_stencil = 0, nnz_stencil = 0;
};
// Builds the layout from the assembled operator A (rows and columns in the
// caller's DOF order) and the lattice coordinates lat [n x 3] of its DOFs
// (-1: off the lattice).  Returns false (and leaves *L empty) when fewer than
// min_fraction of the rows are stencil rows.
bool lattice_layout(const HostCSR &A, const int32_t *lat, int32_t lat_n, double min_fraction, HostLattice *L);

// Element blocks of translated copies of one lattice-aligned cell differ only
// by rounding (their prolongation rows were evaluated at different absolute
// coordinates, their children summed in a different order).  Cells whose DOFs
// all lie on the lattice lat [n_dof x 3] are grouped by the lattice pattern of
// their DOFs; a block that agrees with its group's first block to tol times
// that block's largest entry is replaced by it (in its own local order), so
// that translated rows assemble to equal values.  Returns the number of blocks
// replaced.
int64_t canonical_blocks(const HostCells &C, const int32_t *lat, HostBlocks &K, double tol);

// max_i sum_j |a_ij| / sqrt(a_ii a_jj): Gershgorin bound of D^-1/2 A D^-1/2,
// which has the spectrum of D^-1 A and stays bounded by the row length for
// symmetric positive semi-definite A even where some a_ii are tiny.
double gershgorin_scaled(const HostCSR &A);

// Floating components of a symmetric matrix graph: connected components whose
// rows sum to ~0 (pure-Neumann constants).  Returns per-row id or -1.
std::vector<int32_t> floating_components(const HostCSR &A, int32_t *n_comp);

}  // namespace fvem
