// C ABI, hierarchy setup and the MG-PCG driver of the FastVEM solver.
//
// Solve (paper Sec. 3.1 "solve K p = r", preconditioned per Sec. 4):
//   b = B u (projected divergence, Sec. 3.2), zero mean on pure-Neumann
//   components; FP64 flexible PCG (Polak-Ribiere beta, x0 = 0, true-residual
//   replacement every m iterations, stop on ||b - K x|| / ||b|| <= tol);
//   preconditioner: one V(1,1) cycle of the Galerkin hierarchy with
//   degree-5 Chebyshev smoothing of D^-1 A over [lmax/30, lmax], restriction
//   R = P^T, prolong-and-correct, and a dense semi-definite Cholesky
//   generalised inverse on the coarsest level.  In the mixed mode the
//   V-cycle's operators and vectors are FP32 and the coarsest solve FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fvem.h"
#include "kernels.hpp"
#include "transport.hpp"
#include "elem.hpp"
#include "grid.hpp"
#include "setup_host.hpp"
#include "progress.hpp"

namespace fvem {

static thread_local std::string g_last_error;

#define HIPCHECK(call)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) {                                                                         \
      if (e_ == hipErrorOutOfMemory)                                                                \
        throw SetupError{FVEM_ERR_OOM, std::string(#call) + ": " + hipGetErrorString(e_)};           \
      throw SetupError{FVEM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};             \
    }                                                                                               \
  } while (0)

struct DevMem {
  std::vector<void *> ptrs;
  int64_t bytes = 0;
  template <typename T>
  T *alloc(int64_t n) {
    if (n <= 0) n = 1;
    void *p = nullptr;
    HIPCHECK(hipMalloc(&p, sizeof(T) * n));
    ptrs.push_back(p);
    bytes += sizeof(T) * n;
    return static_cast<T *>(p);
  }
  template <typename T>
  T *upload(const std::vector<T> &v, hipStream_t s) {
    T *p = alloc<T>(static_cast<int64_t>(v.size()));
    if (!v.empty()) HIPCHECK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return p;
  }
  template <typename T>
  T *alloc_zero(int64_t n, hipStream_t s) {
    T *p = alloc<T>(n);
    HIPCHECK(hipMemsetAsync(p, 0, sizeof(T) * std::max<int64_t>(n, 1), s));
    return p;
  }
  ~DevMem() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

// Level operator in the sliced layout; one column array serves both value
// precisions.  Host copies of the slice table and row lengths let the
// operator be read back.
struct DevValues {
  int64_t *vp = nullptr;
  int32_t *tid = nullptr;
  int32_t nt = 0, tw = 0;
  int64_t nvals = 0, nnz_explicit = 0, rows_templated = 0;
};

struct DevSELL {
  int64_t n = 0, m = 0, nnz = 0, nslices = 0;
  int64_t *cp = nullptr, *bt = nullptr;
  int32_t *sl = nullptr;
  int32_t *ci = nullptr, *btab = nullptr;
  uint16_t *c16 = nullptr;
  int64_t n_ci = 0, n_c16 = 0;
  int64_t col_bytes = 0;            // algorithmic column bytes: 2 or 4 per nonzero, 256 per block table
  int64_t slices_coded = 0, slices_plain = 0, slices_templated = 0, slices_stored = 0;
  DevValues d64, d32;               // exact FP64 and single-precision value sets
  double *v64 = nullptr, *tv64 = nullptr;
  float *v32 = nullptr, *tv32 = nullptr;
  std::vector<int64_t> hsp, hcp, hbt;
  std::vector<int32_t> hsl, hrl, hbtab;
  HostValues hv64;                  // FP64 value set without its values (read back on demand)
  bool split = false;
  int32_t *rowmap = nullptr;        // stored row r is output row rowmap[r] (transfers; level 0 with stencil)
  std::vector<int32_t> hrowmap;
  // lattice stencil rows (level 0 when the descriptor gives lattice coordinates)
  struct Stencil {
    int64_t ntiles = 0, n_rows = 0, nnz = 0;
    int32_t *tiles = nullptr, *tile_base = nullptr, *len = nullptr, *off = nullptr;
    uint64_t *mask = nullptr;
    double *val64 = nullptr, *dinv64 = nullptr;
    float *val32 = nullptr, *dinv32 = nullptr;
    int32_t tn = 0, lat_n = 0;
    bool standard = false;          // every class has the full order-2 support
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // set while the stencil launch is timed
    HostLattice host;               // tables, tiles and masks for read-back
  } st;
  DevSELLView<double> d() const {
    DevSELLView<double> v{n, m, nslices, sl, cp, ci, bt, c16, btab, d64.vp, v64, d64.tid, tv64, d64.tw, split, rowmap};
    v.st = {st.ntiles, st.tiles, st.mask, st.tile_base, st.tn, st.lat_n, st.len, st.off, st.val64, st.dinv64,
            st.standard, st.ev0, st.ev1};
    return v;
  }
  DevSELLView<float> f() const {
    DevSELLView<float> v{n, m, nslices, sl, cp, ci, bt, c16, btab, d32.vp, v32, d32.tid, tv32, d32.tw, split, rowmap};
    v.st = {st.ntiles, st.tiles, st.mask, st.tile_base, st.tn, st.lat_n, st.len, st.off, st.val32, st.dinv32,
            st.standard, st.ev0, st.ev1};
    return v;
  }
};

struct Level {
  int64_t n = 0;      // vector length: DOFs, or lattice slots with holes and then the rest
  int64_t ndof = 0;   // the level's DOFs
  DevSELL A;
  DevSELL P, R;   // transfers in their own length-sorted row order (rowmap)
  std::vector<int32_t> order;   // level order: order[internal] = caller's DOF index
  double *dinv64 = nullptr;
  float *dinv32 = nullptr;
  double lmax = 0;
  std::vector<double> ca, cb;
  double *b64, *x64, *xb64, *d64, *r64;
  float *b32, *x32, *xb32, *d32, *r32;
};

}  // namespace fvem

struct fvem_hierarchy {
  fvem::DevMem mem;
  int device = 0;
  int nlev = 0;
  std::vector<fvem::Level> lv;
  int64_t nvert = 0, n0 = 0;   // n0: the caller's level-0 DOFs
  int64_t nl0 = 0;             // level-0 vector length (lattice slots with holes, then the rest)
  int32_t *perm0 = nullptr, *iperm0 = nullptr;   // level-0 order and its inverse (device)
  // divergence and velocity operators from the level-0 element blocks (cell
  // fields: 12 values per level-0 cell)
  fvem::ElemView el;
  int64_t ncell_v = 0;
  double *vs1 = nullptr, *vs2 = nullptr;
  int32_t *comp0 = nullptr;
  int32_t *compc = nullptr;   // component of each DOF in the caller's order
  int ncomp0 = 0;
  double *scratch = nullptr;  // this device's copy of the static scratch array
  // device bytes by structure: level operators, transfers, level vectors and
  // diagonals, divergence, velocity operators, coarsest inverse, PCG workspace
  int64_t mem_by_kind[7] = {0, 0, 0, 0, 0, 0, 0};
  // coarsest level
  int64_t nc = 0;
  double *G = nullptr;
  double *bc = nullptr, *xc = nullptr;
  // PCG
  double *b, *x, *r, *z, *zold, *p, *q, *lam, *partial, *dotout, *mean;
  double *host = nullptr;  // pinned scalars
  std::atomic<int> busy{0};
  // profiling
  std::vector<hipEvent_t> ev;    // pairs around finest-level Chebyshev steps
  size_t ev_used = 0;
  std::vector<hipEvent_t> evv;   // pairs around V-cycles
  size_t evv_used = 0;
  std::vector<hipEvent_t> evs;   // pairs around the stencil launches of finest Chebyshev steps
  size_t evs_used = 0;
  bool profiling = false;         // HIP events around the finest-level launches (V-cycles run eagerly)
  bool profile_vcycle = false;    // HIP events around every V-cycle
  // V-cycles as HIP graphs: one per precision and buffer state (smoothing
  // swaps each level's x buffers an odd number of times, so consecutive
  // V-cycles alternate between two pointer states)
  struct VGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<void *> before, after;   // level buffer pointers at capture and after it
  };
  bool use_graphs = true;
  hipStream_t gstream = nullptr;         // capture and replay stream (default priority)
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  VGraph vg[4];                          // [precision][state]
};

namespace fvem {

static void check(bool ok, const std::string &msg) {
  if (!ok) throw SetupError{FVEM_ERR_INVALID, msg};
}

static bool finite_all(const double *v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

static HostCells cells_of(const fvem_level_desc &L, int64_t n_dof, const char *what) {
  check(L.n_cells >= 0 && (L.n_cells == 0 || (L.cell_ptr && L.cell_dof)), std::string(what) + ": cell arrays");
  HostCells c;
  c.n_cells = L.n_cells;
  c.ptr.assign(L.cell_ptr, L.cell_ptr + L.n_cells + 1);
  check(c.ptr[0] == 0, std::string(what) + ": cell_ptr[0] != 0");
  for (int64_t i = 0; i < L.n_cells; ++i) check(c.ptr[i + 1] >= c.ptr[i], std::string(what) + ": cell_ptr not monotone");
  c.dof.assign(L.cell_dof, L.cell_dof + c.ptr[L.n_cells]);
  for (int32_t d : c.dof) check(d >= -1 && d < n_dof, std::string(what) + ": cell DOF index out of range");
  return c;
}

static HostCSR csr_of(const fvem_csr &M, int64_t rows, int64_t cols, const char *what) {
  check(M.n_rows == rows && M.n_cols == cols, std::string(what) + ": shape mismatch");
  check(M.row_ptr && (M.nnz == 0 || (M.col && M.val)), std::string(what) + ": null arrays");
  HostCSR A;
  A.n_rows = rows;
  A.n_cols = cols;
  A.rp.assign(M.row_ptr, M.row_ptr + rows + 1);
  check(A.rp[0] == 0 && A.rp[rows] == M.nnz, std::string(what) + ": row_ptr ends");
  for (int64_t i = 0; i < rows; ++i) check(A.rp[i + 1] >= A.rp[i], std::string(what) + ": row_ptr not monotone");
  A.ci.assign(M.col, M.col + M.nnz);
  A.v.assign(M.val, M.val + M.nnz);
  for (int32_t j : A.ci) check(j >= 0 && j < cols, std::string(what) + ": column out of range");
  check(finite_all(A.v.data(), M.nnz), std::string(what) + ": non-finite value");
  return A;
}


static DevSELL upload_sell(fvem_hierarchy *h, const HostCSR &A, int max_templates, bool codes, hipStream_t s) {
  HostSELL S = to_sell(A, max_templates > 0, 64, std::max(max_templates, 1), codes);
  DevSELL d;
  d.n = S.n;
  d.m = S.m;
  d.nnz = S.nnz;
  d.nslices = S.nslices;
  d.cp = h->mem.upload(S.cp, s);
  d.bt = h->mem.upload(S.bt, s);
  d.sl = h->mem.upload(S.sl, s);
  d.ci = h->mem.upload(S.ci, s);
  d.c16 = h->mem.upload(S.c16, s);
  d.btab = h->mem.upload(S.btab, s);
  d.n_ci = static_cast<int64_t>(S.ci.size());
  d.n_c16 = static_cast<int64_t>(S.c16.size());
  for (int64_t sl = 0; sl < S.nslices; ++sl) {
    int64_t e = 0;
    for (int64_t i = 64 * sl; i < std::min(S.n, 64 * sl + 64); ++i) e += S.rl[i];
    d.col_bytes += S.bt[sl] >= 0 ? 2 * e + 256 : 4 * e;
  }
  auto meta = [&](const HostValues &V, DevValues &D) {
    D.vp = h->mem.upload(V.vp, s);
    D.tid = h->mem.upload(V.tid, s);
    D.nt = V.nt;
    D.tw = V.tw;
    D.nvals = static_cast<int64_t>(V.v.size());
    D.nnz_explicit = V.nnz_explicit;
    D.rows_templated = V.rows_templated;
  };
  meta(S.v64, d.d64);
  meta(S.v32, d.d32);
  d.v64 = h->mem.upload(S.v64.v, s);
  d.tv64 = h->mem.upload(S.v64.tv, s);
  {
    // FP32 values: cast on the device through a temporary FP64 copy
    DevMem tmp;
    double *t = tmp.upload(S.v32.v, s);
    d.v32 = h->mem.alloc<float>(d.d32.nvals);
    cast_f64_f32(d.d32.nvals, t, d.v32, s);
    double *tt = tmp.upload(S.v32.tv, s);
    d.tv32 = h->mem.alloc<float>(static_cast<int64_t>(S.v32.tv.size()));
    cast_f64_f32(static_cast<int64_t>(S.v32.tv.size()), tt, d.tv32, s);
    HIPCHECK(hipStreamSynchronize(s));   // before the temporaries and host arrays go
  }
  for (int64_t k = 0; k < S.nslices; ++k) {
    (S.bt[k] >= 0 ? d.slices_coded : d.slices_plain) += 1;
    (S.v32.vp[k] < 0 ? d.slices_templated : d.slices_stored) += 1;
  }
  d.hsp = std::move(S.sp);
  d.hcp = std::move(S.cp);
  d.hbt = std::move(S.bt);
  d.hbtab = std::move(S.btab);
  d.hsl = std::move(S.sl);
  d.hrl = std::move(S.rl);
  d.hv64 = std::move(S.v64);
  HostValues().v.swap(d.hv64.v);
  return d;
}

// A level on the lattice layout: the stencil rows go to the class tables,
// every other row (off the lattice, or not matching its class's stencil)
// to sliced storage in its own length-sorted order with a row map into the
// padded level order.  A is in the caller's order; inv maps caller DOF ->
// level slot.
// Rows are sorted by length inside windows of this many rows before they are
// cut into 64-row slices (sliced storage pads each slice to its longest
// row).  A narrower window keeps a slice's rows, and so the x values they
// gather, closer together; a wider one pads less.  On the 128^3 plates,
// windows of 256, 384, 512, 768, 1024 and 4096 rows gave 2.34, 2.37, 2.40,
// 2.40, 2.33 and 2.33 solves/s, and 64 (no sorting across slices) 2.03.
constexpr int64_t ORDER_WINDOW = 512;
// Operators small enough for the row-split kernel, where 16 lanes share a
// row and a wavefront covers only 4 rows, keep 4096-row windows (2.41 ->
// 2.44 solves/s on the same workload).
static int64_t order_window(int64_t n_rows, int64_t small_rows) {
  return small_rows >= 0 && n_rows <= small_rows ? 4096 : ORDER_WINDOW;
}

static void upload_lattice_level(fvem_hierarchy *h, Level &V, const HostCSR &A, HostLattice &lat,
                                 const std::vector<int32_t> &inv, int max_templates, bool codes, int64_t small_rows,
                                 hipStream_t s) {
  std::vector<int32_t> rest;   // caller DOFs of the sliced rows, in level order
  for (int64_t r = 0; r < static_cast<int64_t>(V.order.size()); ++r) {
    const int32_t i = V.order[r];
    if (i >= 0 && !lat.is_stencil[i]) rest.push_back(i);
  }
  const HostCSR R0 = permute(A, rest, &inv, V.n);
  const std::vector<int32_t> ord = window_order(R0, ORDER_WINDOW);
  V.A = upload_sell(h, permute(R0, ord, nullptr, V.n), max_templates, codes, s);
  std::vector<int32_t> rowmap(ord.size());
  for (size_t k = 0; k < ord.size(); ++k) rowmap[k] = inv[rest[ord[k]]];
  V.A.rowmap = h->mem.upload(rowmap, s);
  V.A.hrowmap = std::move(rowmap);
  // the sliced rows share lanes like a small level's when there are few of them
  V.A.split = small_rows >= 0 && static_cast<int64_t>(ord.size()) <= small_rows;
  V.A.m = V.n;
  auto &st = V.A.st;
  st.ntiles = static_cast<int64_t>(lat.tiles.size());
  st.n_rows = lat.n_stencil;
  st.nnz = lat.nnz_stencil;
  st.tn = lat.tn;
  st.lat_n = lat.lat_n;
  st.tiles = h->mem.upload(lat.tiles, s);
  st.mask = h->mem.upload(lat.mask, s);
  st.tile_base = h->mem.upload(lat.tile_base, s);
  const std::vector<int32_t> lens(lat.len, lat.len + 8);
  st.len = h->mem.upload(lens, s);
  st.off = h->mem.upload(lat.off, s);
  st.val64 = h->mem.upload(lat.val, s);
  // the unrolled kernel applies when every class has the standard order-2
  // support: offsets in [-2, 2] along even and [-1, 1] along odd coordinates
  st.standard = true;
  for (int t = 0; t < 8 && st.standard; ++t) {
    const int ra = (t >> 2) ? 1 : 2, rb = ((t >> 1) & 1) ? 1 : 2, rc = (t & 1) ? 1 : 2;
    int j = 0;
    for (int da = -ra; da <= ra && st.standard; ++da)
      for (int db = -rb; db <= rb && st.standard; ++db)
        for (int dc = -rc; dc <= rc && st.standard; ++dc, ++j)
          st.standard = j < lat.len[t] && lat.delta[128 * t + j] == (da + 2) * 25 + (db + 2) * 5 + (dc + 2);
    st.standard = st.standard && j == lat.len[t];
  }
  st.val32 = h->mem.alloc<float>(static_cast<int64_t>(lat.val.size()));
  cast_f64_f32(static_cast<int64_t>(lat.val.size()), st.val64, st.val32, s);
  {
    // every stencil row of a class has the class's diagonal (offset code 62:
    // zero offset), so its D^-1 is the class's: 1 / a_ii as for the vector
    std::vector<double> dv(8, 0.0);
    for (int t = 0; t < 8; ++t)
      for (int j = 0; j < lat.len[t]; ++j)
        if (lat.delta[128 * t + j] == 62 && lat.val[128 * t + j] > 0.0) dv[t] = 1.0 / lat.val[128 * t + j];
    st.dinv64 = h->mem.upload(dv, s);
    st.dinv32 = h->mem.alloc<float>(8);
    cast_f64_f32(8, st.dinv64, st.dinv32, s);
  }
  HIPCHECK(hipStreamSynchronize(s));
  lat.order.clear();
  lat.order.shrink_to_fit();
  lat.is_stencil.clear();
  lat.is_stencil.shrink_to_fit();
  st.host = std::move(lat);
}

static std::vector<int32_t> inverse(const std::vector<int32_t> &order, int64_t n = -1) {
  std::vector<int32_t> inv(n >= 0 ? static_cast<size_t>(n) : order.size(), -1);
  for (size_t i = 0; i < order.size(); ++i)
    if (order[i] >= 0) inv[order[i]] = static_cast<int32_t>(i);
  return inv;
}

// Level-0 operators applied from their element blocks (divergence B and, with
// vc_off, the velocity operators): index lists per cell in the level order,
// the descriptor's block arrays as given (cells of one shape share a block),
// and the positions of every pressure slot and vertex among the cells'
// lists, in increasing order, for the summation of shared outputs.
static void build_elem(fvem_hierarchy *h, const fvem_grid_desc *g, const HostCells &c0,
                       const std::vector<int32_t> &inv0, hipStream_t s) {
  const int64_t nc = c0.n_cells, nv = g->n_vert, nl = h->nl0;
  ElemView &E = h->el;
  E.ncell = nc;
  E.nl = nl;
  E.nv = nv;
  std::vector<int64_t> vptr(g->cell_vptr, g->cell_vptr + nc + 1);
  std::vector<int32_t> vert(g->cell_vert, g->cell_vert + vptr[nc]);
  std::vector<int32_t> cdof(c0.dof.size());
  for (size_t e = 0; e < c0.dof.size(); ++e) cdof[e] = c0.dof[e] >= 0 ? inv0[c0.dof[e]] : -1;
  // positions of each pressure slot among cdof and of each vertex among vert
  std::vector<int64_t> pptr(nl + 1, 0), qptr(nv + 1, 0);
  for (int32_t d : cdof)
    if (d >= 0) pptr[d + 1]++;
  for (int32_t v : vert) qptr[v + 1]++;
  for (int64_t i = 0; i < nl; ++i) pptr[i + 1] += pptr[i];
  for (int64_t i = 0; i < nv; ++i) qptr[i + 1] += qptr[i];
  check(pptr[nl] < (int64_t(1) << 31) && static_cast<int64_t>(cdof.size()) < (int64_t(1) << 31) &&
            3 * static_cast<int64_t>(vert.size()) < (int64_t(1) << 31),
        "cell index lists too long for int32 positions");
  std::vector<int32_t> ppos(pptr[nl]), qpos(qptr[nv]);
  {
    std::vector<int64_t> fp(pptr.begin(), pptr.end() - 1), fq(qptr.begin(), qptr.end() - 1);
    for (size_t e = 0; e < cdof.size(); ++e)
      if (cdof[e] >= 0) ppos[fp[cdof[e]]++] = static_cast<int32_t>(e);
    for (size_t e = 0; e < vert.size(); ++e) qpos[fq[vert[e]]++] = static_cast<int32_t>(e);
  }
  int64_t mark = h->mem.bytes;
  E.cptr = h->mem.upload(c0.ptr, s);
  E.cdof = h->mem.upload(cdof, s);
  E.vptr = h->mem.upload(vptr, s);
  E.vert = h->mem.upload(vert, s);
  E.pptr = h->mem.upload(pptr, s);
  E.ppos = h->mem.upload(ppos, s);
  E.qptr = h->mem.upload(qptr, s);
  E.qpos = h->mem.upload(qpos, s);
  E.tmp = h->mem.alloc<double>(std::max<int64_t>(static_cast<int64_t>(cdof.size()), 3 * vptr[nc]));
  std::vector<int64_t> be_off(g->be_off, g->be_off + nc);
  std::vector<double> be_val(g->be_val, g->be_val + g->be_len);
  E.be_off = h->mem.upload(be_off, s);
  E.be_val = h->mem.upload(be_val, s);
  h->mem_by_kind[3] += h->mem.bytes - mark;
  if (g->vc_off) {
    mark = h->mem.bytes;
    check(g->vc_val && g->vc_len >= 0 && g->cell_geom && g->vert_xyz, "velocity data incomplete");
    check(finite_all(g->vc_val, g->vc_len), "velocity blocks: non-finite value");
    check(finite_all(g->cell_geom, 5 * nc), "cell geometry: non-finite value");
    check(finite_all(g->vert_xyz, 3 * nv), "vertex coordinates: non-finite value");
    std::vector<double> W(nv, 0.0);   // volume around each vertex
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t nvE = vptr[c + 1] - vptr[c], nE = c0.ptr[c + 1] - c0.ptr[c];
      check(g->vc_off[c] >= 0 && g->vc_off[c] + 4 * nvE + 12 * nE + 16 <= g->vc_len, "velocity block out of range");
      check(g->cell_geom[5 * c + 3] > 0 && g->cell_geom[5 * c + 4] > 0, "cell diameter or volume not positive");
      for (int64_t q = vptr[c]; q < vptr[c + 1]; ++q) W[vert[q]] += g->cell_geom[5 * c + 4];
    }
    std::vector<double> winv(nv, 0.0);
    for (int64_t v = 0; v < nv; ++v) winv[v] = W[v] > 0 ? 1.0 / W[v] : 0.0;
    std::vector<int64_t> vc_off(g->vc_off, g->vc_off + nc);
    std::vector<double> vc_val(g->vc_val, g->vc_val + g->vc_len), geom(g->cell_geom, g->cell_geom + 5 * nc),
        xyz(g->vert_xyz, g->vert_xyz + 3 * nv);
    E.vc_off = h->mem.upload(vc_off, s);
    E.vc_val = h->mem.upload(vc_val, s);
    E.geom = h->mem.upload(geom, s);
    E.xyz = h->mem.upload(xyz, s);
    E.winv = h->mem.upload(winv, s);
    h->ncell_v = nc;
    h->vs1 = h->mem.alloc<double>(12 * nc);
    h->vs2 = h->mem.alloc<double>(12 * nc);
    h->mem_by_kind[4] += h->mem.bytes - mark;
  }
  HIPCHECK(hipStreamSynchronize(s));   // the host arrays are temporaries
  progress("hierarchy: element operators stored");
}

static void cheb_coefficients(Level &L, int deg, double lower) {
  const double hi = L.lmax, lo = lower * L.lmax;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  L.ca.assign(deg, 0.0);
  L.cb.assign(deg, 0.0);
  L.cb[0] = 1.0 / theta;
  for (int j = 1; j < deg; ++j) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    L.ca[j] = rn * rho;
    L.cb[j] = 2.0 * rn / delta;
    rho = rn;
  }
}

// ---------------------------------------------------------------- static scratch
//
// Scratch of the entry point that allocates nothing (fvem_project_noalloc):
// the per-block partial sums and means of the component projection for up to
// NOALLOC_MAX_COMP components.  One copy per device, alive until the process
// ends.  In host code the array's name is not a device address: its address
// on each device comes from hipGetSymbolAddress, taken once per device with
// that device current (at the first hierarchy build on it).
constexpr int NOALLOC_MAX_COMP = 16;
constexpr int64_t NOALLOC_PARTIAL = 2 * static_cast<int64_t>(NOALLOC_MAX_COMP) * REDUCE_BLOCKS;
static __device__ __align__(256) double scratch[NOALLOC_PARTIAL + NOALLOC_MAX_COMP];

static double *static_scratch_address(int device) {
  static std::mutex mu;
  static std::vector<double *> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) throw SetupError{FVEM_ERR_INVALID, "bad device id"};
  if (static_cast<size_t>(device) >= addr.size()) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw SetupError{FVEM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    addr[device] = static_cast<double *>(p);
  }
  return addr[device];
}

// Translated coarse element blocks that agree to this fraction of their
// largest entry are one block up to rounding: an entry of P_f^T K_f P_f sums
// at most 27 x 27 products per child over 8 children (k = 2), so two
// evaluation orders differ by at most about 5832 unit roundoffs (6.5e-13) of
// the summed magnitudes.
constexpr double CANONICAL_TOL = 1e-12;

static void build(fvem_hierarchy *h, const fvem_grid_desc *g, const fvem_options *o, hipStream_t s) {
  check(g != nullptr, "null descriptor");
  check(g->n_levels >= 1 && g->levels, "n_levels < 1");
  const int L = g->n_levels;
  const int deg = (o && o->cheb_degree > 0) ? o->cheb_degree : 5;
  const double lower = (o && o->cheb_lower > 0) ? o->cheb_lower : 1.0 / 30.0;
  const int64_t dense_max = (o && o->coarse_dense_max > 0) ? o->coarse_dense_max : 16384;
  const double rcond = (o && o->coarse_rcond > 0) ? o->coarse_rcond : 0.0;
  const double shift = (o && o->coarse_shift > 0) ? o->coarse_shift : 1e-8;
  const int64_t small_rows = (o && o->small_level_rows != 0) ? o->small_level_rows : 400000;
  const int max_templates = (o && o->max_templates != 0) ? o->max_templates : 4096;
  const double lattice_min = (o && o->lattice_min_fraction != 0) ? o->lattice_min_fraction : 0.5;
  const bool general = o && o->galerkin_general != 0;
  h->use_graphs = !(o && o->vcycle_graphs < 0);
  const bool codes = !(o && o->column_codes < 0);
  HIPCHECK(hipGetDevice(&h->device));
  h->nlev = L;
  h->lv.resize(L);
  std::vector<HostCells> cells(L);
  for (int l = 0; l < L; ++l) {
    check(g->levels[l].n_dof >= 0 && g->levels[l].n_dof < (int64_t(1) << 31), "n_dof out of range");
    cells[l] = cells_of(g->levels[l], g->levels[l].n_dof, "level cells");
  }
  for (int l = 0; l + 1 < L; ++l) {
    check(g->levels[l].parent != nullptr, "parent map missing");
    for (int64_t c = 0; c < cells[l].n_cells; ++c)
      check(g->levels[l].parent[c] >= 0 && g->levels[l].parent[c] < cells[l + 1].n_cells, "parent out of range");
  }
  // level-0 element stiffness blocks
  const HostCells &c0 = cells[0];
  HostBlocks ke;
  check(g->ke_off && g->ke_val && g->ke_len >= 0, "element stiffness missing");
  ke.off.assign(g->ke_off, g->ke_off + c0.n_cells);
  for (int64_t c = 0; c < c0.n_cells; ++c) {
    const int64_t m = c0.ptr[c + 1] - c0.ptr[c];
    check(ke.off[c] >= 0 && ke.off[c] + m * m <= g->ke_len, "element stiffness block out of range");
  }
  ke.val.assign(g->ke_val, g->ke_val + g->ke_len);
  check(finite_all(ke.val.data(), g->ke_len), "element stiffness: non-finite value");
  h->n0 = g->levels[0].n_dof;
  // divergence
  h->nvert = g->n_vert;
  check(g->n_vert >= 0, "n_vert");
  if (g->n_vert > 0) {
    check(g->cell_vptr && g->cell_vert && g->be_off && g->be_val && g->be_len >= 0, "divergence blocks missing");
    check(g->cell_vptr[0] == 0, "cell_vptr[0] must be 0");
    for (int64_t c = 0; c < c0.n_cells; ++c) {
      check(g->cell_vptr[c + 1] >= g->cell_vptr[c], "cell_vptr not increasing");
      for (int64_t k = g->cell_vptr[c]; k < g->cell_vptr[c + 1]; ++k)
        check(g->cell_vert[k] >= 0 && g->cell_vert[k] < g->n_vert, "cell vertex out of range");
      const int64_t w = 3 * (g->cell_vptr[c + 1] - g->cell_vptr[c]);
      check(g->be_off[c] >= 0 && g->be_off[c] + (c0.ptr[c + 1] - c0.ptr[c]) * w <= g->be_len,
            "divergence block out of range");
    }
    check(finite_all(g->be_val, g->be_len), "divergence: non-finite value");
  }
  // components of level 0
  std::vector<int32_t> comp0(h->n0, -1);
  if (g->component) comp0.assign(g->component, g->component + h->n0);
  h->ncomp0 = g->n_components;
  for (int32_t c : comp0) check(c >= -1 && c < h->ncomp0, "component id out of range");

  // operators per level: A_0 from element blocks, A_{l+1} element-wise Galerkin
  std::vector<HostCSR> A(L), P(L);
  A[0] = assemble_blocks(h->n0, h->n0, c0, c0, ke);
  progress("hierarchy: level 0 assembled, n=%lld nnz=%lld", static_cast<long long>(A[0].n_rows),
           static_cast<long long>(A[0].rp.back()));
  if (general) {
    // prolongations that may reach beyond one coarse cell: A_{l+1} = P^T A_l P
    // by sparse products on the host
    for (int l = 0; l + 1 < L; ++l) {
      P[l] = csr_of(g->levels[l].P, g->levels[l].n_dof, g->levels[l + 1].n_dof, "prolongation");
      A[l + 1] = galerkin_product(A[l], P[l]);
      progress("hierarchy: sparse Galerkin level %d, n=%lld nnz=%lld", l + 1,
               static_cast<long long>(A[l + 1].n_rows), static_cast<long long>(A[l + 1].nnz()));
    }
    HostBlocks().val.swap(ke.val);
  }
  // element-wise Galerkin products on the device; the coarse blocks stay
  // resident as the next level's fine blocks
  auto kmem = std::make_unique<DevMem>();
  const int64_t *kfoff = kmem->upload(ke.off, s);
  const double *kf = kmem->upload(ke.val, s);
  HIPCHECK(hipStreamSynchronize(s));
  { HostBlocks().val.swap(ke.val); }
  for (int l = 0; l + 1 < L && !general; ++l) {
    const int64_t nf = g->levels[l].n_dof, nc = g->levels[l + 1].n_dof;
    P[l] = csr_of(g->levels[l].P, nf, nc, "prolongation");
    const HostCells &F = cells[l], &C = cells[l + 1];
    const int64_t ncc = C.n_cells;
    // children of each coarse cell in increasing order; block offsets; staging
    std::vector<int64_t> chptr(ncc + 1, 0), child(F.n_cells), ooff(ncc + 1, 0), soff(ncc, -1);
    for (int64_t f = 0; f < F.n_cells; ++f) chptr[g->levels[l].parent[f] + 1]++;
    for (int64_t c = 0; c < ncc; ++c) chptr[c + 1] += chptr[c];
    {
      std::vector<int64_t> fill(chptr.begin(), chptr.end() - 1);
      for (int64_t f = 0; f < F.n_cells; ++f) child[fill[g->levels[l].parent[f]]++] = f;
    }
    for (int64_t c = 0; c < ncc; ++c) {
      const int64_t m = C.ptr[c + 1] - C.ptr[c];
      ooff[c + 1] = ooff[c] + m * m;
    }
    // cells whose K_f, P_f and T do not fit the LDS buffer stage in global
    // scratch; launches are cut into batches of at most 2^26 scratch doubles
    constexpr int64_t SCRATCH_CAP = int64_t(1) << 26;
    std::vector<std::pair<int64_t, int64_t>> batches;   // [c0, c1)
    int64_t need_max = 0, b0 = 0, used = 0;
    for (int64_t c = 0; c < ncc; ++c) {
      const int64_t m = C.ptr[c + 1] - C.ptr[c];
      int64_t mf = 0;
      for (int64_t q = chptr[c]; q < chptr[c + 1]; ++q) mf = std::max(mf, F.ptr[child[q] + 1] - F.ptr[child[q]]);
      const int64_t need = mf * mf + 2 * mf * m;
      if (need > GALERKIN_LDS_DOUBLES) {
        check(need <= SCRATCH_CAP, "coarse cell too large for the Galerkin staging buffer");
        if (used + need > SCRATCH_CAP) {
          batches.emplace_back(b0, c);
          b0 = c;
          used = 0;
        }
        soff[c] = used;
        used += need;
        need_max = std::max(need_max, used);
      }
    }
    batches.emplace_back(b0, ncc);
    DevMem tmp;
    const int64_t *d_fptr = tmp.upload(F.ptr, s);
    const int32_t *d_fdof = tmp.upload(F.dof, s);
    const int64_t *d_prp = tmp.upload(P[l].rp, s);
    const int32_t *d_pci = tmp.upload(P[l].ci, s);
    const double *d_pv = tmp.upload(P[l].v, s);
    const int64_t *d_cptr = tmp.upload(C.ptr, s);
    const int32_t *d_cdof = tmp.upload(C.dof, s);
    const int64_t *d_chptr = tmp.upload(chptr, s);
    const int64_t *d_child = tmp.upload(child, s);
    const int64_t *d_soff = tmp.upload(soff, s);
    double *scratch = tmp.alloc<double>(std::max<int64_t>(need_max, 1));
    int *bad = tmp.alloc<int>(1);
    const int big = 0x7fffffff;
    HIPCHECK(hipMemcpyAsync(bad, &big, sizeof(int), hipMemcpyHostToDevice, s));
    auto knew = std::make_unique<DevMem>();
    const int64_t *d_ooff = knew->upload(ooff, s);
    double *d_out = knew->alloc<double>(std::max<int64_t>(ooff[ncc], 1));
    HIPCHECK(hipMemsetAsync(d_out, 0, sizeof(double) * std::max<int64_t>(ooff[ncc], 1), s));
    for (const auto &bt : batches)
      galerkin(bt.first, bt.second - bt.first, d_fptr, d_fdof, kfoff, kf, d_prp, d_pci, d_pv, d_cptr, d_cdof,
               d_chptr, d_child, d_ooff, d_out, d_soff, scratch, bad, s);
    int hbad = big;
    HIPCHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HostBlocks knext;
    knext.off.assign(ooff.begin(), ooff.end() - 1);
    knext.val.resize(ooff[ncc]);
    if (ooff[ncc]) HIPCHECK(hipMemcpyAsync(knext.val.data(), d_out, sizeof(double) * ooff[ncc], hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (hbad != big)
      throw SetupError{FVEM_ERR_INVALID, "prolongation row " + std::to_string(hbad) +
                                             " references a DOF outside the parent cell (not diffusion-free)"};
    if (g->levels[l + 1].dof_lattice && l + 2 < L) {
      // translated copies of a lattice-aligned coarse cell get one block, so
      // that their rows assemble to equal values (stencil rows); done
      // whether or not the level then takes the lattice layout, so that both
      // layouts hold one operator
      const int64_t nrep = canonical_blocks(C, g->levels[l + 1].dof_lattice, knext, CANONICAL_TOL);
      if (nrep && ooff[ncc])
        HIPCHECK(hipMemcpyAsync(d_out, knext.val.data(), sizeof(double) * ooff[ncc], hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
      progress("hierarchy: level %d, %lld translated element blocks made identical", l + 1,
               static_cast<long long>(nrep));
    }
    A[l + 1] = assemble_blocks(nc, nc, C, C, knext);
    progress("hierarchy: Galerkin level %d, n=%lld nnz=%lld", l + 1, static_cast<long long>(nc),
             static_cast<long long>(A[l + 1].rp.back()));
    kmem = std::move(knew);
    kfoff = d_ooff;
    kf = d_out;
  }
  kmem.reset();

  // level order: rows sorted by length inside windows (order_window); every
  // level operator, transfer and per-DOF array is renumbered into it
  std::vector<std::vector<int32_t>> inv(L);
  // a level below the coarsest takes the lattice layout when the
  // descriptor gives its lattice coordinates and enough of its rows are
  // stencil rows; its order is then the padded lattice order (slots with
  // holes, then the DOFs off the lattice) and A stays in the caller's order
  std::vector<HostLattice> lat(L);
  std::vector<char> on_lattice(L, 0);
  for (int l = 0; l + 1 < L; ++l) {
    const fvem_level_desc &ld = g->levels[l];
    if (!ld.dof_lattice || ld.lattice_n <= 0 || lattice_min < 0) continue;
    on_lattice[l] = lattice_layout(A[l], ld.dof_lattice, ld.lattice_n, lattice_min, &lat[l]);
    if (on_lattice[l])
      progress("hierarchy: level %d lattice layout, %lld of %lld rows on stencils, %lld tiles", l,
               static_cast<long long>(lat[l].n_stencil), static_cast<long long>(A[l].n_rows),
               static_cast<long long>(lat[l].tiles.size()));
  }
  for (int l = 0; l < L; ++l) {
    h->lv[l].ndof = A[l].n_rows;
    if (on_lattice[l]) {
      h->lv[l].order = lat[l].order;
      inv[l] = inverse(lat[l].order, A[l].n_rows);
      continue;
    }
    h->lv[l].order = window_order(A[l], order_window(A[l].n_rows, small_rows));
    inv[l] = inverse(h->lv[l].order);
    A[l] = permute(A[l], h->lv[l].order, &inv[l]);
  }
  h->nl0 = static_cast<int64_t>(h->lv[0].order.size());
  for (int l = 0; l + 1 < L; ++l)
    P[l] = permute(P[l], h->lv[l].order, &inv[l + 1], static_cast<int64_t>(h->lv[l + 1].order.size()));
  std::vector<int32_t> comp_caller = comp0;
  {
    std::vector<int32_t> c(h->nl0, -1);
    for (int64_t i = 0; i < h->nl0; ++i)
      if (h->lv[0].order[i] >= 0) c[i] = comp0[h->lv[0].order[i]];
    comp0.swap(c);
  }
  h->perm0 = h->mem.upload(h->lv[0].order, s);
  h->iperm0 = h->mem.upload(inv[0], s);
  progress("hierarchy: level order and renumbering done");

  // upload
  for (int l = 0; l < L; ++l) {
    Level &V = h->lv[l];
    std::vector<double> dinv;
    int64_t mark = h->mem.bytes;
    if (on_lattice[l]) {
      V.n = static_cast<int64_t>(V.order.size());
      upload_lattice_level(h, V, A[l], lat[l], inv[l], max_templates, codes, small_rows, s);
      dinv.assign(V.n, 0.0);
      const HostCSR &Al = A[l];
#pragma omp parallel for schedule(dynamic, 4096)
      for (int64_t r = 0; r < V.n; ++r) {
        const int32_t i = V.order[r];
        if (i < 0) continue;
        double d = 0.0;
        for (int64_t k = Al.rp[i]; k < Al.rp[i + 1]; ++k)
          if (Al.ci[k] == i) d = Al.v[k];
        dinv[r] = d > 0.0 ? 1.0 / d : 0.0;
      }
    } else {
      V.n = A[l].n_rows;
      const bool split = small_rows >= 0 && V.n <= small_rows;
      V.A = upload_sell(h, A[l], max_templates, codes, s);
      V.A.split = split;
      dinv.assign(V.n, 0.0);
      for (int64_t i = 0; i < V.n; ++i) {
        double d = 0.0;
        for (int64_t k = A[l].rp[i]; k < A[l].rp[i + 1]; ++k)
          if (A[l].ci[k] == i) d = A[l].v[k];
        dinv[i] = d > 0.0 ? 1.0 / d : 0.0;
      }
    }
    h->mem_by_kind[0] += h->mem.bytes - mark;
    mark = h->mem.bytes;
    V.dinv64 = h->mem.upload(dinv, s);
    V.dinv32 = h->mem.alloc<float>(V.n);
    cast_f64_f32(V.n, V.dinv64, V.dinv32, s);
    V.lmax = gershgorin_scaled(A[l]);
    cheb_coefficients(V, deg, lower);
    h->mem_by_kind[2] += h->mem.bytes - mark;
    mark = h->mem.bytes;
    if (l + 1 < L) {
      // transfers: rows sorted by length inside windows (own order), values
      // from templates where rows repeat; outputs are scattered back by rowmap
      auto transfer = [&](const HostCSR &T) {
        const std::vector<int32_t> ord = window_order(T, order_window(T.n_rows, small_rows));
        const bool split = small_rows >= 0 && T.n_rows <= small_rows;
        DevSELL d = upload_sell(h, permute(T, ord, nullptr), max_templates, codes, s);
        d.rowmap = h->mem.upload(ord, s);
        d.split = split;
        HIPCHECK(hipStreamSynchronize(s));
        return d;
      };
      V.P = transfer(P[l]);
      V.R = transfer(transpose(P[l]));
    }
    h->mem_by_kind[1] += h->mem.bytes - mark;
    mark = h->mem.bytes;
    progress("hierarchy: level %d stored (%lld of %lld rows templated)", l,
             static_cast<long long>(V.A.d32.rows_templated), static_cast<long long>(V.n));
    // level vectors start at zero: lattice holes are never written and stay zero
    V.b64 = h->mem.alloc_zero<double>(V.n, s);
    V.x64 = h->mem.alloc_zero<double>(V.n, s);
    V.xb64 = h->mem.alloc_zero<double>(V.n, s);
    V.d64 = h->mem.alloc_zero<double>(V.n, s);
    V.r64 = h->mem.alloc_zero<double>(V.n, s);
    V.b32 = h->mem.alloc_zero<float>(V.n, s);
    V.x32 = h->mem.alloc_zero<float>(V.n, s);
    V.xb32 = h->mem.alloc_zero<float>(V.n, s);
    V.d32 = h->mem.alloc_zero<float>(V.n, s);
    V.r32 = h->mem.alloc_zero<float>(V.n, s);
    h->mem_by_kind[2] += h->mem.bytes - mark;
    if (l + 1 < L) A[l] = HostCSR();   // the coarsest stays for the dense factorisation
  }
  h->comp0 = h->mem.upload(comp0, s);
  h->compc = h->mem.upload(comp_caller, s);
  h->scratch = static_scratch_address(h->device);
  if (g->n_vert > 0) build_elem(h, g, c0, inv[0], s);
  progress("hierarchy: operators uploaded");

  // coarsest level: dense semi-definite factorisation and generalised inverse
  const HostCSR &Ac = A[L - 1];
  h->nc = Ac.n_rows;
  check(h->nc <= dense_max, "coarsest level exceeds coarse_dense_max");
  {
    const int64_t n = h->nc;
    std::vector<double> diag0(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = Ac.rp[i]; k < Ac.rp[i + 1]; ++k)
        if (Ac.ci[k] == i) diag0[i] = Ac.v[k];
    // A_c is positive semi-definite (pure-Neumann constants; coarse DOF
    // combinations the prolongation annihilates); every restricted
    // right-hand side is orthogonal to those directions, so the coarsest
    // level solves with the positive definite A_c + shift diag(A_c)
    std::vector<double> dshift(n);
    for (int64_t i = 0; i < n; ++i) dshift[i] = shift * diag0[i];
    double *dg = h->mem.upload(diag0, s);
    double *ds = h->mem.upload(dshift, s);
    DevMem tmp;
    double *D = tmp.alloc<double>(n * n);
    double *X = tmp.alloc<double>(n * n);
    int *flag = tmp.alloc<int>(1);
    HIPCHECK(hipMemsetAsync(flag, 0, sizeof(int), s));
    int64_t *crp = tmp.alloc<int64_t>(n + 1);
    int32_t *cci = tmp.alloc<int32_t>(Ac.nnz());
    double *cv = tmp.alloc<double>(Ac.nnz());
    HIPCHECK(hipMemcpyAsync(crp, Ac.rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(cci, Ac.ci.data(), sizeof(int32_t) * Ac.nnz(), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(cv, Ac.v.data(), sizeof(double) * Ac.nnz(), hipMemcpyHostToDevice, s));
    dense_from_csr(n, crp, cci, cv, D, s);
    add_diagonal(n, D, ds, s);
    potrf_semidefinite(D, n, dg, rcond, flag, s);
    trinv_semidefinite(D, X, n, s);
    h->G = h->mem.alloc<double>(n * n);
    h->mem_by_kind[5] += static_cast<int64_t>(sizeof(double)) * n * n;
    // G = X^T X
    gemm_f64(n, n, n, 1.0, X, n, 1, X, 1, n, 0.0, h->G, n, false, s);
    int hflag = 0;
    HIPCHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (hflag) throw SetupError{FVEM_ERR_NOT_SPD, "coarsest operator is not positive semi-definite"};
    progress("hierarchy: coarsest level factorised, n=%lld", static_cast<long long>(n));
    h->bc = h->mem.alloc<double>(n);
    h->xc = h->mem.alloc<double>(n);
  }
  // PCG workspace (level-0 vector length, zero holes)
  const int64_t n = h->nl0;
  const int64_t mark_pcg = h->mem.bytes;
  h->b = h->mem.alloc_zero<double>(n, s);
  h->x = h->mem.alloc_zero<double>(n, s);
  h->r = h->mem.alloc_zero<double>(n, s);
  h->z = h->mem.alloc_zero<double>(n, s);
  h->zold = h->mem.alloc_zero<double>(n, s);
  h->p = h->mem.alloc_zero<double>(n, s);
  h->q = h->mem.alloc_zero<double>(n, s);
  h->partial = h->mem.alloc<double>(2 * MAX_COMP * REDUCE_BLOCKS);
  h->dotout = h->mem.alloc<double>(8);
  h->mean = h->mem.alloc<double>(MAX_COMP);
  h->lam = h->mem.alloc_zero<double>(n, s);
  HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&h->host), 8 * sizeof(double), hipHostMallocDefault));
  h->mem_by_kind[6] += h->mem.bytes - mark_pcg;
  HIPCHECK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- V-cycle

template <typename T> struct Vec;
template <> struct Vec<double> {
  static double *b(Level &L) { return L.b64; }
  static double *&x(Level &L) { return L.x64; }
  static double *&xb(Level &L) { return L.xb64; }
  static double *d(Level &L) { return L.d64; }
  static double *r(Level &L) { return L.r64; }
  static const double *dinv(Level &L) { return L.dinv64; }
  static DevSELLView<double> A(Level &L) { return L.A.d(); }
  static DevSELLView<double> P(Level &L) { return L.P.d(); }
  static DevSELLView<double> R(Level &L) { return L.R.d(); }
};
template <> struct Vec<float> {
  static float *b(Level &L) { return L.b32; }
  static float *&x(Level &L) { return L.x32; }
  static float *&xb(Level &L) { return L.xb32; }
  static float *d(Level &L) { return L.d32; }
  static float *r(Level &L) { return L.r32; }
  static const float *dinv(Level &L) { return L.dinv32; }
  static DevSELLView<float> A(Level &L) { return L.A.f(); }
  static DevSELLView<float> P(Level &L) { return L.P.f(); }
  static DevSELLView<float> R(Level &L) { return L.R.f(); }
};

static void ev_record(std::vector<hipEvent_t> &ev, size_t &used, hipStream_t s) {
  if (used == ev.size()) {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    ev.push_back(e);
  }
  HIPCHECK(hipEventRecord(ev[used++], s));
}
static void ev_record(fvem_hierarchy *h, hipStream_t s) { ev_record(h->ev, h->ev_used, s); }

template <typename T>
static void coarse_solve(fvem_hierarchy *h, hipStream_t s) {
  Level &C = h->lv[h->nlev - 1];
  const int64_t n = h->nc;
  if constexpr (sizeof(T) == 4) {
    cast_scale(n, C.b32, h->bc, 1.0, s);
  } else {
    HIPCHECK(hipMemcpyAsync(h->bc, C.b64, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  symv(n, h->G, h->bc, h->xc, s);
  if constexpr (sizeof(T) == 4) {
    cast_scale(n, h->xc, C.x32, 1.0, s);
  } else {
    HIPCHECK(hipMemcpyAsync(C.x64, h->xc, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
}

template <typename T>
static void smooth(fvem_hierarchy *h, int l, bool from_zero, hipStream_t s) {
  Level &L = h->lv[l];
  using V = Vec<T>;
  const int deg = static_cast<int>(L.ca.size());
  int j0 = 0;
  if (from_zero) {
    cheb_first<T>(L.n, V::b(L), V::dinv(L), V::d(L), V::x(L), static_cast<T>(L.cb[0]), s);
    j0 = 1;
  }
  for (int j = j0; j < deg; ++j) {
    const bool prof = h->profiling && l == 0;
    if (prof) {
      ev_record(h, s);
      if (L.A.st.ntiles > 0) {
        // the stencil launch inside the step is timed on its own
        while (h->evs.size() < h->evs_used + 2) {
          hipEvent_t e;
          HIPCHECK(hipEventCreate(&e));
          h->evs.push_back(e);
        }
        L.A.st.ev0 = h->evs[h->evs_used++];
        L.A.st.ev1 = h->evs[h->evs_used++];
      }
    }
    cheb_step<T>(V::A(L), V::b(L), V::dinv(L), V::x(L), V::d(L), V::xb(L), static_cast<T>(L.ca[j]),
                 static_cast<T>(L.cb[j]), s);
    if (prof) {
      ev_record(h, s);
      L.A.st.ev0 = L.A.st.ev1 = nullptr;
    }
    std::swap(V::x(L), V::xb(L));
  }
}

template <typename T>
static void vcycle(fvem_hierarchy *h, int l, hipStream_t s) {
  if (l == h->nlev - 1) {
    coarse_solve<T>(h, s);
    return;
  }
  using V = Vec<T>;
  Level &L = h->lv[l];
  Level &N = h->lv[l + 1];
  smooth<T>(h, l, true, s);
  residual<T>(V::A(L), V::x(L), V::b(L), V::r(L), s);
  spmv<T>(V::R(L), V::r(L), V::b(N), s);
  vcycle<T>(h, l + 1, s);
  spmv_add<T>(V::P(L), V::x(N), V::x(L), s);
  smooth<T>(h, l, false, s);
}

// pointers of every level's smoothing buffers of precision T (the state a
// V-cycle's graph was captured in; each precision has its own buffers)
template <typename T>
static std::vector<void *> vcycle_state(fvem_hierarchy *h) {
  std::vector<void *> v;
  for (Level &L : h->lv) {
    v.push_back(Vec<T>::x(L));
    v.push_back(Vec<T>::xb(L));
  }
  return v;
}

template <typename T>
static void set_vcycle_state(fvem_hierarchy *h, const std::vector<void *> &v) {
  size_t k = 0;
  for (Level &L : h->lv) {
    Vec<T>::x(L) = static_cast<T *>(v[k++]);
    Vec<T>::xb(L) = static_cast<T *>(v[k++]);
  }
}

// One V-cycle on stream s.  Unprofiled V-cycles run as HIP graphs: the
// first in each buffer state is captured on the hierarchy's own stream and
// replayed from then on; events join that stream to s both ways.  No node
// is a memset (fills are kernels).  A failed capture switches graphs off for
// the handle and runs the V-cycle eagerly.
template <typename T>
static void run_vcycle(fvem_hierarchy *h, hipStream_t s) {
  if (!h->use_graphs || h->profiling) {
    vcycle<T>(h, 0, s);
    return;
  }
  const std::vector<void *> cur = vcycle_state<T>(h);
  const int base = sizeof(T) == 8 ? 2 : 0;
  fvem_hierarchy::VGraph *g = nullptr;
  for (int k = 0; k < 2 && !g; ++k)
    if (h->vg[base + k].exec && h->vg[base + k].before == cur) g = &h->vg[base + k];
  if (!h->gstream) {
    HIPCHECK(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&h->gev_in, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&h->gev_out, hipEventDisableTiming));
  }
  if (!g) {
    fvem_hierarchy::VGraph *slot = !h->vg[base].exec ? &h->vg[base] : !h->vg[base + 1].exec ? &h->vg[base + 1] : nullptr;
    if (!slot) throw SetupError{FVEM_ERR_HIP, "V-cycle graph: unexpected buffer state"};
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      try {
        vcycle<T>(h, 0, h->gstream);
      } catch (...) {
        ok = false;
      }
      ok = hipStreamEndCapture(h->gstream, &graph) == hipSuccess && ok && graph;
    }
    hipGraphExec_t exec = nullptr;
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {
      h->use_graphs = false;
      set_vcycle_state<T>(h, cur);
      vcycle<T>(h, 0, s);
      return;
    }
    slot->exec = exec;
    slot->before = cur;
    slot->after = vcycle_state<T>(h);
    g = slot;
  }
  HIPCHECK(hipEventRecord(h->gev_in, s));
  HIPCHECK(hipStreamWaitEvent(h->gstream, h->gev_in, 0));
  HIPCHECK(hipGraphLaunch(g->exec, h->gstream));
  HIPCHECK(hipEventRecord(h->gev_out, h->gstream));
  HIPCHECK(hipStreamWaitEvent(s, h->gev_out, 0));
  set_vcycle_state<T>(h, g->after);
}

// z = M r (level-0 input r, FP64), projected
static void precondition(fvem_hierarchy *h, const double *r, double *z, bool mixed, double rnorm, hipStream_t s) {
  Level &L0 = h->lv[0];
  const int64_t n = h->nl0;
  if (h->nlev == 1) {
    symv(n, h->G, r, z, s);
  } else if (mixed) {
    const double sc = rnorm > 0 ? 1.0 / rnorm : 1.0;
    cast_scale(n, r, L0.b32, sc, s);
    if (h->profile_vcycle) ev_record(h->evv, h->evv_used, s);
    run_vcycle<float>(h, s);
    if (h->profile_vcycle) ev_record(h->evv, h->evv_used, s);
    cast_scale(n, L0.x32, z, 1.0 / sc, s);
  } else {
    HIPCHECK(hipMemcpyAsync(L0.b64, r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (h->profile_vcycle) ev_record(h->evv, h->evv_used, s);
    run_vcycle<double>(h, s);
    if (h->profile_vcycle) ev_record(h->evv, h->evv_used, s);
    HIPCHECK(hipMemcpyAsync(z, L0.x64, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  if (h->ncomp0) project_components(n, z, h->comp0, h->ncomp0, h->partial, h->mean, s);
}

static void dots_host_n(fvem_hierarchy *h, int64_t n, int nd, const double *a0, const double *b0, const double *a1,
                        const double *b1, const double *a2, const double *b2, double *out, hipStream_t s) {
  dots(n, nd, a0, b0, a1, b1, a2, b2, h->partial, h->dotout, s);
  HIPCHECK(hipMemcpyAsync(h->host, h->dotout, sizeof(double) * nd, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int j = 0; j < nd; ++j) out[j] = h->host[j];
}

static void dots_host(fvem_hierarchy *h, int nd, const double *a0, const double *b0, const double *a1,
                      const double *b1, const double *a2, const double *b2, double *out, hipStream_t s) {
  dots(h->nl0, nd, a0, b0, a1, b1, a2, b2, h->partial, h->dotout, s);
  HIPCHECK(hipMemcpyAsync(h->host, h->dotout, sizeof(double) * nd, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int j = 0; j < nd; ++j) out[j] = h->host[j];
}

static fvem_status pcg(fvem_hierarchy *h, const double *bin, double *xout, const fvem_solve_opts *so,
                       fvem_solve_stats *st, hipStream_t s) {
  const int64_t n = h->nl0;
  const double tol = (so && so->tol > 0) ? so->tol : 1e-8;
  const int maxit = (so && so->maxit > 0) ? so->maxit : 500;
  const bool mixed = so && so->precision == FVEM_PREC_MIXED;
  const int m = (so && so->replace_every > 0) ? so->replace_every : 10;
  const DevSELLView<double> K = h->lv[0].A.d();
  HIPCHECK(hipMemcpyAsync(h->b, bin, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (h->ncomp0) project_components(n, h->b, h->comp0, h->ncomp0, h->partial, h->mean, s);
  double d[3];
  dots_host(h, 1, h->b, h->b, nullptr, nullptr, nullptr, nullptr, d, s);
  const double bb = d[0];
  if (!std::isfinite(bb)) throw SetupError{FVEM_ERR_NONFINITE, "non-finite right-hand side"};
  fill<double>(n, h->x, 0.0, s);
  if (bb == 0.0) {
    HIPCHECK(hipMemcpyAsync(xout, h->x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (st) { st->iterations = 0; st->rel_residual = 0.0; }
    return FVEM_OK;
  }
  const double nb = std::sqrt(bb);
  HIPCHECK(hipMemcpyAsync(h->r, h->b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  precondition(h, h->r, h->z, mixed, nb, s);
  HIPCHECK(hipMemcpyAsync(h->p, h->z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  // PCG scalars stay on the device: sc[0..1] and sc[4..5] hold (r.z, r.z_old)
  // of alternate iterations, sc[2] = p.Kp, sc[3] = r.r.  alpha and beta are
  // formed by the update kernels from them; the host waits once per
  // iteration, for r.r (the stopping test) together with p.Kp and r.z.
  double *sc = h->dotout;
  int cur = 0;   // slot of the current r.z
  dots(n, 1, h->r, h->z, nullptr, nullptr, nullptr, nullptr, h->partial, sc + cur, s);
  int it = 0;
  double rel = 1.0;
  fvem_status status = FVEM_ERR_NOT_CONVERGED;
  while (it < maxit) {
    spmv<double>(K, h->p, h->q, s);
    dots(n, 1, h->p, h->q, nullptr, nullptr, nullptr, nullptr, h->partial, sc + 2, s);
    pcg_update_xr(n, sc + cur, sc + 2, h->p, h->q, h->x, h->r, s);
    ++it;
    if (it % m == 0) residual<double>(K, h->x, h->b, h->r, s);
    dots(n, 1, h->r, h->r, nullptr, nullptr, nullptr, nullptr, h->partial, sc + 3, s);
    HIPCHECK(hipMemcpyAsync(h->host, sc, sizeof(double) * 6, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double rz = h->host[cur], pq = h->host[2];
    if (!(pq > 0.0) || !std::isfinite(rz)) throw SetupError{FVEM_ERR_NONFINITE, "CG breakdown (p.Kp <= 0)"};
    d[0] = h->host[3];
    rel = std::sqrt(d[0]) / nb;
    if (rel <= tol) {
      // the true residual decides (slot 6: the r.z slots stay live)
      residual<double>(K, h->x, h->b, h->r, s);
      dots(n, 1, h->r, h->r, nullptr, nullptr, nullptr, nullptr, h->partial, sc + 6, s);
      HIPCHECK(hipMemcpyAsync(h->host + 6, sc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      d[0] = h->host[6];
      rel = std::sqrt(d[0]) / nb;
      if (rel <= tol) {
        status = FVEM_OK;
        break;
      }
    }
    if (it >= maxit) break;
    std::swap(h->z, h->zold);
    precondition(h, h->r, h->z, mixed, std::sqrt(d[0]), s);
    const int nxt = 4 - cur;
    dots(n, 2, h->r, h->z, h->r, h->zold, nullptr, nullptr, h->partial, sc + nxt, s);
    // beta = (r.z - r.z_old) / (previous r.z), Polak-Ribiere
    pcg_update_p(n, h->z, sc + nxt, sc + nxt + 1, sc + cur, h->p, s);
    cur = nxt;
  }
  if (status != FVEM_OK) {
    residual<double>(K, h->x, h->b, h->r, s);
    dots_host(h, 1, h->r, h->r, nullptr, nullptr, nullptr, nullptr, d, s);
    rel = std::sqrt(d[0]) / nb;
    char buf[96];
    std::snprintf(buf, sizeof buf, "maxit = %d reached at relative residual %.3e", static_cast<int>(maxit), rel);
    g_last_error = buf;
  }
  if (h->ncomp0) project_components(n, h->x, h->comp0, h->ncomp0, h->partial, h->mean, s);
  HIPCHECK(hipMemcpyAsync(xout, h->x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (st) {
    st->iterations = it;
    st->rel_residual = rel;
  }
  return status;
}

enum SolveKind { SOLVE_FORWARD, SOLVE_ADJOINT, SOLVE_VELOCITY, SOLVE_VELOCITY_ADJOINT };

// One solve with timing and stats.  SOLVE_VELOCITY: out = s = Pi_1 u -
// grad Pi_k p (p also to p_out unless null); SOLVE_VELOCITY_ADJOINT:
// out = g_u = Pi_1^T g_s + B^T K^+ (-(grad Pi_k)^T g_s).
static fvem_status solve_common(fvem_hierarchy *h, const double *in, double *out, const fvem_solve_opts *so,
                                fvem_solve_stats *st, hipStream_t s, SolveKind kind, double *p_out = nullptr) {
  const bool adjoint = kind == SOLVE_ADJOINT;
  const bool vel_op = kind == SOLVE_VELOCITY || kind == SOLVE_VELOCITY_ADJOINT;
  const bool velocity = vel_op || !so || so->input == FVEM_INPUT_VELOCITY;
  if (velocity && h->nvert == 0) throw SetupError{FVEM_ERR_INVALID, "no divergence operator in this hierarchy"};
  if (vel_op && h->ncell_v == 0) throw SetupError{FVEM_ERR_INVALID, "no velocity operators in this hierarchy"};
  h->profiling = so && so->profile == 1;
  h->profile_vcycle = so && so->profile != 0;
  h->ev_used = 0;
  h->evv_used = 0;
  h->evs_used = 0;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  HIPCHECK(hipEventRecord(e0, s));
  // caller's DOF order <-> level order at the boundary of the solve
  const int64_t n = h->n0, nl = h->nl0;
  fvem_status stt;
  if (kind == SOLVE_VELOCITY) {
    elem_apply(h->el, ELEM_B, in, h->q, false, 1.0, s);
    stt = pcg(h, h->q, h->lam, so, st, s);
    if (p_out) gather(n, h->iperm0, h->lam, p_out, s);
    elem_apply(h->el, ELEM_PI, in, out, false, 1.0, s);
    elem_apply(h->el, ELEM_G, h->lam, out, true, -1.0, s);   // s = Pi_1 u - G p
  } else if (kind == SOLVE_VELOCITY_ADJOINT) {
    elem_apply(h->el, ELEM_GT, in, h->q, false, -1.0, s);   // g_p = -G^T g_s (level order)
    stt = pcg(h, h->q, h->lam, so, st, s);
    elem_apply(h->el, ELEM_BT, h->lam, out, false, 1.0, s);
    elem_apply(h->el, ELEM_PIT, in, out, true, 1.0, s);
  } else if (!adjoint) {
    const double *rhs = h->q;
    if (velocity) elem_apply(h->el, ELEM_B, in, h->q, false, 1.0, s);
    else gather(nl, h->perm0, in, h->q, s);
    stt = pcg(h, rhs, h->lam, so, st, s);
    gather(n, h->iperm0, h->lam, out, s);
  } else {
    gather(nl, h->perm0, in, h->q, s);
    stt = pcg(h, h->q, h->lam, so, st, s);
    if (velocity) elem_apply(h->el, ELEM_BT, h->lam, out, false, 1.0, s);
    else gather(n, h->iperm0, h->lam, out, s);
  }
  HIPCHECK(hipEventRecord(e1, s));
  HIPCHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    st->ms_total = ms;
    st->n_levels = h->nlev;
    st->ms_fine_smoother = 0.0;
    st->n_fine_smoother = static_cast<int32_t>(h->ev_used / 2);
    for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, h->ev[k], h->ev[k + 1]));
      st->ms_fine_smoother += t;
    }
    st->ms_fine_stencil = 0.0;
    st->n_fine_stencil = static_cast<int32_t>(h->evs_used / 2);
    for (size_t k = 0; k + 1 < h->evs_used; k += 2) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, h->evs[k], h->evs[k + 1]));
      st->ms_fine_stencil += t;
    }
    st->ms_vcycle = 0.0;
    st->n_vcycle = static_cast<int32_t>(h->evv_used / 2);
    for (size_t k = 0; k + 1 < h->evv_used; k += 2) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, h->evv[k], h->evv[k + 1]));
      st->ms_vcycle += t;
    }
  }
  h->profiling = false;
  h->profile_vcycle = false;
  return stt;
}

template <typename F>
static fvem_status guard(F &&f) {
  try {
    return f();
  } catch (const SetupError &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return FVEM_ERR_OOM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return FVEM_ERR_INVALID;
  }
}

struct BusyGuard {
  fvem_hierarchy *h;
  bool ok;
  explicit BusyGuard(fvem_hierarchy *hh) : h(hh) {
    int z = 0;
    ok = h->busy.compare_exchange_strong(z, 1);
  }
  ~BusyGuard() {
    if (ok) h->busy.store(0);
  }
};

}  // namespace fvem

using namespace fvem;

extern "C" {

fvem_status fvem_hierarchy_build(const fvem_grid_desc *g, const fvem_options *o, void *hip_stream,
                                 fvem_hierarchy **out) {
  if (!out) {
    g_last_error = "null output handle";
    return FVEM_ERR_INVALID;
  }
  *out = nullptr;
  fvem_hierarchy *h = new (std::nothrow) fvem_hierarchy();
  if (!h) return FVEM_ERR_OOM;
  fvem_status st = guard([&] {
    build(h, g, o, static_cast<hipStream_t>(hip_stream));
    return FVEM_OK;
  });
  if (st != FVEM_OK) {
    delete h;
    return st;
  }
  *out = h;
  return FVEM_OK;
}

fvem_status fvem_solve(fvem_hierarchy *h, const double *in_dev, double *p_dev, const fvem_solve_opts *so,
                       fvem_solve_stats *st, void *hip_stream) {
  if (!h || !in_dev || !p_dev) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  BusyGuard bg(h);
  if (!bg.ok) {
    g_last_error = "another solve is running on this handle";
    return FVEM_ERR_BUSY;
  }
  return guard([&] { return solve_common(h, in_dev, p_dev, so, st, static_cast<hipStream_t>(hip_stream), SOLVE_FORWARD); });
}

fvem_status fvem_solve_adjoint(fvem_hierarchy *h, const double *gp_dev, double *gu_dev, const fvem_solve_opts *so,
                               fvem_solve_stats *st, void *hip_stream) {
  if (!h || !gp_dev || !gu_dev) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  BusyGuard bg(h);
  if (!bg.ok) {
    g_last_error = "another solve is running on this handle";
    return FVEM_ERR_BUSY;
  }
  return guard([&] { return solve_common(h, gp_dev, gu_dev, so, st, static_cast<hipStream_t>(hip_stream), SOLVE_ADJOINT); });
}

fvem_status fvem_project_velocity(fvem_hierarchy *h, const double *u_dev, double *s_dev, double *p_dev,
                                  const fvem_solve_opts *so, fvem_solve_stats *st, void *hip_stream) {
  if (!h || !u_dev || !s_dev) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  BusyGuard bg(h);
  if (!bg.ok) {
    g_last_error = "another solve is running on this handle";
    return FVEM_ERR_BUSY;
  }
  return guard([&] {
    return solve_common(h, u_dev, s_dev, so, st, static_cast<hipStream_t>(hip_stream), SOLVE_VELOCITY, p_dev);
  });
}

fvem_status fvem_project_velocity_adjoint(fvem_hierarchy *h, const double *gs_dev, double *gu_dev,
                                          const fvem_solve_opts *so, fvem_solve_stats *st, void *hip_stream) {
  if (!h || !gs_dev || !gu_dev) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  BusyGuard bg(h);
  if (!bg.ok) {
    g_last_error = "another solve is running on this handle";
    return FVEM_ERR_BUSY;
  }
  return guard([&] {
    return solve_common(h, gs_dev, gu_dev, so, st, static_cast<hipStream_t>(hip_stream), SOLVE_VELOCITY_ADJOINT);
  });
}

fvem_status fvem_velocity_loss(fvem_hierarchy *h, const double *s_dev, const double *t_dev, double scale,
                               double *loss_host, double *gs_dev, void *hip_stream) {
  if (!h || !s_dev || !t_dev || !loss_host) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  BusyGuard bg(h);
  if (!bg.ok) {
    g_last_error = "another call is running on this handle";
    return FVEM_ERR_BUSY;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  return guard([&] {
    check(h->ncell_v > 0, "no velocity operators in this hierarchy");
    const int64_t m = 12 * h->ncell_v;
    lincomb(m, 1.0, s_dev, -1.0, t_dev, h->vs1, s);     // d = s - t
    elem_apply(h->el, ELEM_M, h->vs1, h->vs2, false, 1.0, s);   // w = M d
    double d[1];
    dots_host_n(h, m, 1, h->vs1, h->vs2, nullptr, nullptr, nullptr, nullptr, d, s);
    if (!std::isfinite(d[0])) throw SetupError{FVEM_ERR_NONFINITE, "non-finite loss"};
    *loss_host = d[0];
    if (gs_dev) {
      lincomb(m, 2.0 * scale, h->vs2, 0.0, nullptr, gs_dev, s);
      HIPCHECK(hipStreamSynchronize(s));
    }
    return FVEM_OK;
  });
}

fvem_status fvem_level_storage(fvem_hierarchy *h, int32_t level, int64_t *nnz, int64_t *nnz_explicit,
                               int64_t *rows_templated, int32_t *n_templates, int32_t *template_width) {
  if (!h || level < 0 || level >= h->nlev) {
    g_last_error = "bad handle or level";
    return FVEM_ERR_INVALID;
  }
  const DevSELL &A = h->lv[level].A;
  if (nnz) *nnz = A.nnz + A.st.nnz;
  if (nnz_explicit) *nnz_explicit = A.d32.nnz_explicit;
  if (rows_templated) *rows_templated = A.d32.rows_templated + A.st.n_rows;
  if (n_templates) *n_templates = A.d32.nt;
  if (template_width) *template_width = A.d32.tw;
  return FVEM_OK;
}

// matrix bytes one application of a sliced operator reads (see fvem_level_bytes)
static int64_t sell_bytes(const DevSELL &A, int32_t precision) {
  const DevValues &V = precision == FVEM_PREC_FP64 ? A.d64 : A.d32;
  const int64_t vb = precision == FVEM_PREC_FP64 ? 8 : 4;
  return A.col_bytes + vb * V.nnz_explicit + 4 * V.rows_templated + 68 * A.st.ntiles +
         (A.rowmap ? 4 * A.n : 0);
}

fvem_status fvem_level_bytes(fvem_hierarchy *h, int32_t level, int32_t precision, int64_t *bytes) {
  if (!h || level < 0 || level >= h->nlev || !bytes) {
    g_last_error = "bad handle, level or output";
    return FVEM_ERR_INVALID;
  }
  // stencil rows: a tile id and 8 mask words per launched tile; sliced
  // rows with a row map: 4 bytes per row
  *bytes = sell_bytes(h->lv[level].A, precision);
  return FVEM_OK;
}

fvem_status fvem_transfer_storage(fvem_hierarchy *h, int32_t level, int32_t precision, int64_t *nnz,
                                  int64_t *bytes_p, int64_t *bytes_r) {
  if (!h || level < 0 || level + 1 >= h->nlev) {
    g_last_error = "bad handle or level (transfers exist below the coarsest level)";
    return FVEM_ERR_INVALID;
  }
  const Level &L = h->lv[level];
  if (nnz) *nnz = L.P.nnz;
  if (bytes_p) *bytes_p = sell_bytes(L.P, precision);
  if (bytes_r) *bytes_r = sell_bytes(L.R, precision);
  return FVEM_OK;
}

fvem_status fvem_vcycle_bytes(fvem_hierarchy *h, int32_t precision, int64_t *bytes) {
  if (!h || !bytes) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  const int64_t s = precision == FVEM_PREC_FP64 ? 8 : 4;
  int64_t total = 0;
  for (int l = 0; l + 1 < h->nlev; ++l) {
    const Level &L = h->lv[l];
    const int64_t n = L.ndof, nn = h->lv[l + 1].ndof;
    const int64_t deg = static_cast<int64_t>(L.ca.size());
    // 2 deg applications of A_l (deg - 1 pre-smoothing steps after the
    // first, the residual, deg post-smoothing steps); vectors: the first
    // step (b, D^-1 read; d, x written), 2 deg - 1 fused steps (x, b, D^-1,
    // d read; d, x written), the residual (x, b read; r written), the
    // restriction (r read, b_c written) and the prolongation (x_c read,
    // x read and written)
    total += 2 * deg * sell_bytes(L.A, precision) + sell_bytes(L.R, precision) + sell_bytes(L.P, precision);
    total += s * (n * (4 + 6 * (2 * deg - 1) + 3 + 1 + 2) + 2 * nn);
    total -= s * (2 * deg - 1) * L.A.st.n_rows;   // stencil rows take D^-1 from their class
  }
  // coarsest: the dense generalised inverse, read once, and its vectors
  total += 8 * h->nc * h->nc + (s + 8) * 2 * h->nc;
  *bytes = total;
  return FVEM_OK;
}

fvem_status fvem_memory_breakdown(fvem_hierarchy *h, int64_t *bytes) {
  if (!h || !bytes) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  for (int k = 0; k < 7; ++k) bytes[k] = h->mem_by_kind[k];
  bytes[7] = h->mem.bytes;
  return FVEM_OK;
}

fvem_status fvem_level_slices(fvem_hierarchy *h, int32_t level, int64_t *coded, int64_t *plain,
                              int64_t *templated, int64_t *stored) {
  if (!h || level < 0 || level >= h->nlev) {
    g_last_error = "bad handle or level";
    return FVEM_ERR_INVALID;
  }
  const DevSELL &A = h->lv[level].A;
  if (coded) *coded = A.slices_coded;
  if (plain) *plain = A.slices_plain;
  if (templated) *templated = A.slices_templated;
  if (stored) *stored = A.slices_stored;
  return FVEM_OK;
}

fvem_status fvem_level_stencil(fvem_hierarchy *h, int32_t level, int64_t *rows, int64_t *nnz, int64_t *tiles) {
  if (!h || level < 0 || level >= h->nlev) {
    g_last_error = "bad handle or level";
    return FVEM_ERR_INVALID;
  }
  const DevSELL &A = h->lv[level].A;
  if (rows) *rows = A.st.n_rows;
  if (nnz) *nnz = A.st.nnz;
  if (tiles) *tiles = A.st.ntiles;
  return FVEM_OK;
}

fvem_status fvem_hierarchy_cells(fvem_hierarchy *h, int64_t *n_cells) {
  if (!h || !n_cells) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  *n_cells = h->ncell_v;
  return FVEM_OK;
}

fvem_status fvem_apply(fvem_hierarchy *h, int32_t op, const double *x, double *y, void *hip_stream) {
  if (!h || !x || !y) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  BusyGuard bg(h);
  if (!bg.ok) {
    g_last_error = "another call is running on this handle";
    return FVEM_ERR_BUSY;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool acc = (op & FVEM_APPLY_ACCUMULATE) != 0;
  op &= ~FVEM_APPLY_ACCUMULATE;
  return guard([&] {
    const int64_t n = h->n0, nl = h->nl0;
    if (op >= FVEM_OP_PI1 && op <= FVEM_OP_AVT) check(h->ncell_v > 0, "no velocity operators in this hierarchy");
    if (acc)
      check(op == FVEM_OP_BT || op == FVEM_OP_PI1 || op == FVEM_OP_PI1T || op == FVEM_OP_G || op == FVEM_OP_MASS ||
                op == FVEM_OP_AV || op == FVEM_OP_AVT,
            "accumulation is not available for this operator");
    auto el = [&](ElemOp eo, const double *xx) { elem_apply(h->el, eo, xx, y, acc, 1.0, s); };
    switch (op) {
      case FVEM_OP_PI1: el(ELEM_PI, x); break;
      case FVEM_OP_PI1T: el(ELEM_PIT, x); break;
      case FVEM_OP_G:
        gather(nl, h->perm0, x, h->p, s);
        el(ELEM_G, h->p);
        break;
      case FVEM_OP_GT:
        elem_apply(h->el, ELEM_GT, x, h->q, false, 1.0, s);
        gather(n, h->iperm0, h->q, y, s);
        break;
      case FVEM_OP_MASS: el(ELEM_M, x); break;
      case FVEM_OP_AV: el(ELEM_AV, x); break;
      case FVEM_OP_AVT: el(ELEM_AVT, x); break;
      case FVEM_OP_K:
        gather(nl, h->perm0, x, h->p, s);
        spmv<double>(h->lv[0].A.d(), h->p, h->q, s);
        gather(n, h->iperm0, h->q, y, s);
        break;
      case FVEM_OP_B:
        check(h->nvert > 0, "no divergence operator");
        elem_apply(h->el, ELEM_B, x, h->q, false, 1.0, s);
        gather(n, h->iperm0, h->q, y, s);
        break;
      case FVEM_OP_BT:
        check(h->nvert > 0, "no divergence operator");
        gather(nl, h->perm0, x, h->p, s);
        el(ELEM_BT, h->p);
        break;
      case FVEM_OP_VCYCLE:
      case FVEM_OP_VCYCLE32: {
        gather(nl, h->perm0, x, h->r, s);
        double nr = 1.0;
        if (op == FVEM_OP_VCYCLE32) {
          double d[1];
          dots_host(h, 1, h->r, h->r, nullptr, nullptr, nullptr, nullptr, d, s);
          nr = std::sqrt(d[0]);
        }
        precondition(h, h->r, h->z, op == FVEM_OP_VCYCLE32, nr, s);
        gather(n, h->iperm0, h->z, y, s);
        break;
      }
      case FVEM_OP_PROJECT:
        gather(nl, h->perm0, x, h->z, s);
        if (h->ncomp0) project_components(nl, h->z, h->comp0, h->ncomp0, h->partial, h->mean, s);
        gather(n, h->iperm0, h->z, y, s);
        break;
      default: throw SetupError{FVEM_ERR_INVALID, "unknown operator"};
    }
    HIPCHECK(hipStreamSynchronize(s));
    return FVEM_OK;
  });
}

fvem_status fvem_project_noalloc(fvem_hierarchy *h, const double *x, double *y, void *hip_stream) {
  if (!h || !x || !y) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  if (h->ncomp0 > NOALLOC_MAX_COMP) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "%d pure-Neumann components exceed the static scratch limit of %d",
                  h->ncomp0, NOALLOC_MAX_COMP);
    g_last_error = buf;
    return FVEM_ERR_INVALID;
  }
  if (!h->scratch) {
    g_last_error = "static scratch address unavailable";
    return FVEM_ERR_HIP;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  return guard([&] {
    const int64_t n = h->n0;
    if (x != y) HIPCHECK(hipMemcpyAsync(y, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (h->ncomp0) project_components(n, y, h->compc, h->ncomp0, h->scratch, h->scratch + NOALLOC_PARTIAL, s);
    HIPCHECK(hipGetLastError());
    return FVEM_OK;
  });
}

fvem_status fvem_level_matrix(fvem_hierarchy *h, int32_t level, int64_t *n_rows, int64_t *nnz, int64_t *row_ptr,
                              int32_t *col, double *val) {
  if (!h || level < 0 || level >= h->nlev) {
    g_last_error = "bad handle or level";
    return FVEM_ERR_INVALID;
  }
  return guard([&] {
    const DevSELL &A = h->lv[level].A;
    if (n_rows) *n_rows = h->lv[level].ndof;
    if (nnz) *nnz = A.nnz + A.st.nnz;
    if (!row_ptr && !col && !val) return FVEM_OK;
    // read back the sliced operator and return it in the caller's order
    HostSELL S;
    S.n = A.n;
    S.m = A.m;
    S.nnz = A.nnz;
    S.nslices = A.nslices;
    S.sp = A.hsp;
    S.cp = A.hcp;
    S.bt = A.hbt;
    S.btab = A.hbtab;
    S.sl = A.hsl;
    S.rl = A.hrl;
    S.v64 = A.hv64;
    S.ci.resize(A.n_ci);
    S.c16.resize(A.n_c16);
    S.v64.v.resize(A.d64.nvals);
    if (A.n_ci) HIPCHECK(hipMemcpy(S.ci.data(), A.ci, sizeof(int32_t) * A.n_ci, hipMemcpyDeviceToHost));
    if (A.n_c16) HIPCHECK(hipMemcpy(S.c16.data(), A.c16, sizeof(uint16_t) * A.n_c16, hipMemcpyDeviceToHost));
    if (A.d64.nvals)
      HIPCHECK(hipMemcpy(S.v64.v.data(), A.v64, sizeof(double) * A.d64.nvals, hipMemcpyDeviceToHost));
    const std::vector<int32_t> &order = h->lv[level].order;
    HostCSR Ls = from_sell(S);
    if (!A.hrowmap.empty() || A.st.ntiles > 0) {
      // sliced rows scattered to their level rows, plus the stencil rows
      const int64_t nl = h->lv[level].n;
      const auto &L = A.st.host;
      std::vector<std::vector<std::pair<int32_t, double>>> rows(nl);
      for (int64_t k = 0; k < Ls.n_rows; ++k)
        for (int64_t q = Ls.rp[k]; q < Ls.rp[k + 1]; ++q) rows[A.hrowmap[k]].emplace_back(Ls.ci[q], Ls.v[q]);
      const int tn = L.tn;
      for (size_t b = 0; b < L.tiles.size(); ++b) {
        const int32_t T = L.tiles[b];
        const int Ta = T / (tn * tn), Tb = (T / tn) % tn, Tc = T % tn;
        for (int t = 0; t < 8; ++t)
          for (int lane = 0; lane < 64; ++lane) {
            if (!((L.mask[8 * b + t] >> lane) & 1)) continue;
            const int a0 = 8 * Ta + (t >> 2) + 2 * (lane >> 4), b0 = 8 * Tb + ((t >> 1) & 1) + 2 * ((lane >> 2) & 3),
                      c0 = 8 * Tc + (t & 1) + 2 * (lane & 3);
            auto &row = rows[L.tile_base[T] + 64 * t + lane];
            for (int j = 0; j < L.len[t]; ++j) {
              const int q = L.delta[128 * t + j];
              const int a = a0 + q / 25 - 2, bb = b0 + (q / 5) % 5 - 2, c = c0 + q % 5 - 2;
              const int32_t base = L.tile_base[((a >> 3) * tn + (bb >> 3)) * tn + (c >> 3)];
              const int cls = 4 * (a & 1) + 2 * (bb & 1) + (c & 1);
              row.emplace_back(base + 64 * cls + 16 * ((a & 7) >> 1) + 4 * ((bb & 7) >> 1) + ((c & 7) >> 1),
                               L.val[128 * t + j]);
            }
          }
      }
      HostCSR P;
      P.n_rows = nl;
      P.n_cols = nl;
      P.rp.assign(nl + 1, 0);
      for (int64_t r = 0; r < nl; ++r) P.rp[r + 1] = P.rp[r] + static_cast<int64_t>(rows[r].size());
      P.ci.resize(P.rp[nl]);
      P.v.resize(P.rp[nl]);
      for (int64_t r = 0; r < nl; ++r)
        for (size_t q = 0; q < rows[r].size(); ++q) {
          P.ci[P.rp[r] + q] = rows[r][q].first;
          P.v[P.rp[r] + q] = rows[r][q].second;
        }
      Ls = std::move(P);
    }
    const int64_t ncaller = h->lv[level].ndof;
    const HostCSR C = permute(Ls, inverse(order, ncaller), &order, ncaller);
    if (row_ptr) std::copy(C.rp.begin(), C.rp.end(), row_ptr);
    if (col) std::copy(C.ci.begin(), C.ci.end(), col);
    if (val) std::copy(C.v.begin(), C.v.end(), val);
    return FVEM_OK;
  });
}

fvem_status fvem_hierarchy_info(fvem_hierarchy *h, int32_t *n_levels, int64_t *n_dof0, int64_t *n_vert,
                                int64_t *device_bytes) {
  if (!h) {
    g_last_error = "null handle";
    return FVEM_ERR_INVALID;
  }
  if (n_levels) *n_levels = h->nlev;
  if (n_dof0) *n_dof0 = h->n0;
  if (n_vert) *n_vert = h->nvert;
  if (device_bytes) *device_bytes = h->mem.bytes;
  return FVEM_OK;
}

void fvem_hierarchy_destroy(fvem_hierarchy *h) {
  if (!h) return;
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->evv) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->evs) (void)hipEventDestroy(e);
  for (auto &g : h->vg)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (h->gev_in) (void)hipEventDestroy(h->gev_in);
  if (h->gev_out) (void)hipEventDestroy(h->gev_out);
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  if (h->host) (void)hipHostFree(h->host);
  delete h;
}

const char *fvem_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

struct fvem_grid {
  fvem::grid::Output out;
  std::vector<fvem_level_desc> levels;
  std::vector<double> xflat;
  std::vector<std::vector<int32_t>> lat;   // per level: lattice coordinates of its DOFs (-1: off the lattice)
};

extern "C" {

fvem_status fvem_grid_build(const double *V, int64_t nv, const int32_t *F, int64_t nt, int32_t N, int32_t k,
                            int32_t levels, int32_t dirichlet_top, int64_t coarse_max, fvem_grid **out) {
  return fvem_grid_build_ex(V, nv, F, nt, N, k, levels, dirichlet_top, coarse_max, 0, out);
}

fvem_status fvem_grid_build_ex(const double *V, int64_t nv, const int32_t *F, int64_t nt, int32_t N, int32_t k,
                               int32_t levels, int32_t dirichlet_top, int64_t coarse_max, int32_t flags,
                               fvem_grid **out) {
  if (!out) {
    g_last_error = "null output handle";
    return FVEM_ERR_INVALID;
  }
  *out = nullptr;
  return guard([&] {
    check(N >= 2 && N <= 1024 && (N & (N - 1)) == 0, "N must be a power of two in [2, 1024]");
    check(k == 1 || k == 2, "k must be 1 or 2");
    check(levels >= 1, "levels must be >= 1");
    check(nv >= 0 && nt >= 0 && (nt == 0 || (V && F)), "boundary mesh arrays");
    for (int64_t i = 0; i < 3 * nt; ++i) check(F[i] >= 0 && F[i] < nv, "triangle vertex index out of range");
    for (int64_t i = 0; i < 3 * nv; ++i) check(std::isfinite(V[i]), "non-finite boundary vertex");
    auto g = std::make_unique<fvem_grid>();
    grid::Input in;
    in.V = V;
    in.nv = nv;
    in.F = F;
    in.nt = nt;
    in.N = N;
    in.k = k;
    in.L = levels;
    in.dirichlet = dirichlet_top != 0;
    in.coarse_max = coarse_max > 0 ? coarse_max : 16384;
    check((flags & ~FVEM_GRID_NAIVE_PROLONGATION) == 0, "unknown grid flag");
    in.naive = (flags & FVEM_GRID_NAIVE_PROLONGATION) != 0;
    try {
      grid::build_grid(in, &g->out);
    } catch (const std::runtime_error &e) {
      throw SetupError{FVEM_ERR_INVALID, std::string("grid construction failed: ") + e.what()};
    }
    const auto &o = g->out;
    const int L = static_cast<int>(o.levels.size());
    g->levels.resize(L);
    for (int l = 0; l < L; ++l) {
      fvem_level_desc &d = g->levels[l];
      const auto &lv = o.levels[l];
      d.n_dof = lv.n_dof;
      d.n_cells = lv.n_cells;
      d.cell_ptr = lv.cell_ptr.data();
      d.cell_dof = lv.cell_dof.data();
      d.parent = l + 1 < L ? lv.parent.data() : nullptr;
      d.P = fvem_csr{};
      if (l + 1 < L) {
        const auto &P = o.P[l];
        d.P.n_rows = lv.n_dof;
        d.P.n_cols = o.levels[l + 1].n_dof;
        d.P.nnz = static_cast<int64_t>(P.ci.size());
        d.P.row_ptr = P.rp.data();
        d.P.col = P.ci.data();
        d.P.val = P.v.data();
      }
    }
    // support points on each level's lattice: cells of side 2^l h, the
    // half-lattice of spacing 2^(l-1) h for k = 2 (vertices, edge midpoints,
    // face and cell centres of whole cubes), the vertex lattice for k = 1
    g->lat.resize(L);
    for (int l = 0; l < L; ++l) {
      const auto &lv = o.levels[l];
      const int64_t div = int64_t(1) << l;
      const int64_t steps = (k == 2 ? 2 * int64_t(N) : int64_t(N)) / div;
      if (steps < 2 || (k == 2 ? 2 * int64_t(N) : int64_t(N)) % div) continue;
      const double scale = static_cast<double>(steps);
      const int32_t lat_n = static_cast<int32_t>(steps) + 1;
      std::vector<int32_t> &lat = g->lat[l];
      lat.assign(3 * lv.n_dof, -1);
      for (int64_t i = 0; i < lv.n_dof; ++i) {
        int32_t c[3];
        bool on = true;
        for (int d = 0; d < 3 && on; ++d) {
          const double q = lv.dof_point[3 * i + d] * scale, r = std::nearbyint(q);
          on = std::fabs(q - r) < 1e-7 && r >= 0 && r < lat_n;
          c[d] = static_cast<int32_t>(r);
        }
        if (on)
          for (int d = 0; d < 3; ++d) lat[3 * i + d] = c[d];
      }
      g->levels[l].dof_lattice = lat.data();
      g->levels[l].lattice_n = lat_n;
    }
    g->xflat.resize(3 * o.X.size());
    for (size_t i = 0; i < o.X.size(); ++i) {
      g->xflat[3 * i] = o.X[i].x;
      g->xflat[3 * i + 1] = o.X[i].y;
      g->xflat[3 * i + 2] = o.X[i].z;
    }
    *out = g.release();
    return FVEM_OK;
  });
}

fvem_status fvem_grid_describe(fvem_grid *g, fvem_grid_desc *d) {
  if (!g || !d) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  const auto &o = g->out;
  d->n_levels = static_cast<int32_t>(g->levels.size());
  d->levels = g->levels.data();
  d->ke_off = o.ke_off.data();
  d->ke_val = o.ke_val.data();
  d->ke_len = static_cast<int64_t>(o.ke_val.size());
  d->n_vert = o.n_vert;
  d->cell_vptr = o.cell_vptr.data();
  d->cell_vert = o.cell_vert.data();
  d->be_off = o.be_off.data();
  d->be_val = o.be_val.data();
  d->be_len = static_cast<int64_t>(o.be_val.size());
  d->component = o.component.data();
  d->n_components = o.n_components;
  d->vc_off = o.vc_off.data();
  d->vc_val = o.vc_val.data();
  d->vc_len = static_cast<int64_t>(o.vc_val.size());
  d->cell_geom = o.cell_geom.data();
  d->vert_xyz = g->xflat.data();
  return FVEM_OK;
}

fvem_status fvem_grid_info(fvem_grid *g, const double **vertices, int64_t *n_vert, const double **dof_points,
                           const int8_t **dof_kind, int64_t *n_dof, int64_t *n_trees, int64_t *n_shared) {
  if (!g) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  const auto &o = g->out;
  if (vertices) *vertices = g->xflat.data();
  if (n_vert) *n_vert = o.n_vert;
  if (dof_points) *dof_points = o.dof_point.data();
  if (dof_kind) *dof_kind = o.dof_kind.data();
  if (n_dof) *n_dof = o.levels.empty() ? 0 : o.levels[0].n_dof;
  if (n_trees) *n_trees = o.n_trees;
  if (n_shared) *n_shared = o.n_shared_blocks;
  return FVEM_OK;
}

fvem_status fvem_grid_level_points(fvem_grid *g, int32_t level, const double **dof_points, const int8_t **dof_kind,
                                   int64_t *n_dof) {
  if (!g || level < 0 || level >= static_cast<int32_t>(g->out.levels.size())) {
    g_last_error = "bad grid or level";
    return FVEM_ERR_INVALID;
  }
  const auto &lv = g->out.levels[level];
  if (dof_points) *dof_points = lv.dof_point.data();
  if (dof_kind) *dof_kind = lv.dof_kind.data();
  if (n_dof) *n_dof = lv.n_dof;
  return FVEM_OK;
}

fvem_status fvem_grid_cell_faces(fvem_grid *g, int64_t cell, int32_t *n_faces, int32_t *n_corners,
                                 int32_t *face_len, int32_t *face_vert, int32_t cap_faces, int32_t cap_corners) {
  if (!g || cell < 0 || cell + 1 >= static_cast<int64_t>(g->out.cell_face_ptr.size())) {
    g_last_error = "bad grid or cell";
    return FVEM_ERR_INVALID;
  }
  const auto &o = g->out;
  const int64_t f0 = o.cell_face_ptr[cell], f1 = o.cell_face_ptr[cell + 1];
  const int64_t nf = f1 - f0, nc = o.face_ptr[f1] - o.face_ptr[f0];
  if (n_faces) *n_faces = static_cast<int32_t>(nf);
  if (n_corners) *n_corners = static_cast<int32_t>(nc);
  if (!face_len && !face_vert) return FVEM_OK;
  if (!face_len || !face_vert || cap_faces < nf || cap_corners < nc) {
    g_last_error = "face buffers missing or too small";
    return FVEM_ERR_INVALID;
  }
  for (int64_t f = f0; f < f1; ++f) face_len[f - f0] = static_cast<int32_t>(o.face_ptr[f + 1] - o.face_ptr[f]);
  std::copy(o.face_vert.begin() + o.face_ptr[f0], o.face_vert.begin() + o.face_ptr[f1], face_vert);
  return FVEM_OK;
}

void fvem_grid_destroy(fvem_grid *g) { delete g; }

}  // extern "C"

// ---------------------------------------------------------------- transport
//
// Point location, P2G, G2P and advection on a native grid's finest level
// (Algorithm 1, Sec. 3.2-3.3).  The structure copies the grid's BSP trees,
// triangle lists and cell geometry to the device; P2G scratch grows with the
// particle count.

struct fvem_transport {
  fvem::DevMem mem;
  fvem::TransportView view;
  int device = 0;
  int32_t *cell_count = nullptr, *cell_start = nullptr, *chunk = nullptr;
  int32_t *order = nullptr;
  int64_t order_cap = 0;
  std::unique_ptr<fvem::DevMem> order_mem;
  unsigned long long *vmax = nullptr;
  std::atomic<int> busy{0};
};

namespace fvem {

struct TransportBusy {
  fvem_transport *t;
  bool ok;
  explicit TransportBusy(fvem_transport *tt) : t(tt) {
    int z = 0;
    ok = t->busy.compare_exchange_strong(z, 1);
  }
  ~TransportBusy() {
    if (ok) t->busy.store(0);
  }
};

static void transport_device(const fvem_transport *t) {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  check(dev == t->device, "transport used on another device than the one it was created on");
}

}  // namespace fvem

extern "C" {

fvem_status fvem_transport_create(const fvem_grid *g, void *hip_stream, fvem_transport **out) {
  if (!g || !out) {
    g_last_error = "null argument";
    return FVEM_ERR_INVALID;
  }
  *out = nullptr;
  return guard([&] {
    const auto &o = g->out;
    check(!o.levels.empty() && !o.loc_bg.empty(), "grid has no finest-level locator");
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto t = std::make_unique<fvem_transport>();
    HIPCHECK(hipGetDevice(&t->device));
    int64_t N3 = static_cast<int64_t>(o.loc_bg.size());
    int32_t N = static_cast<int32_t>(std::llround(std::cbrt(static_cast<double>(N3))));
    check(static_cast<int64_t>(N) * N * N == N3, "locator is not N^3");
    TransportView &v = t->view;
    v.N = N;
    v.bg = t->mem.upload(o.loc_bg, s);
    v.tree_root = t->mem.upload(o.loc_tree_root, s);
    v.plane = t->mem.upload(o.loc_plane, s);
    v.child = t->mem.upload(o.loc_child, s);
    v.leaf_cell = t->mem.upload(o.loc_cell, s);
    v.tri_ptr = t->mem.upload(o.tri_ptr, s);
    v.tri_id = t->mem.upload(o.tri_id, s);
    v.tri_xyz = t->mem.upload(o.tri_xyz, s);
    v.cell_geom = t->mem.upload(o.cell_geom, s);
    v.vert_xyz = t->mem.upload(g->xflat, s);
    v.n_vert = o.n_vert;
    t->cell_count = t->mem.alloc<int32_t>(N3 + 1);
    t->cell_start = t->mem.alloc<int32_t>(N3 + 1);
    t->chunk = t->mem.alloc<int32_t>(p2g_chunks(N));
    t->vmax = t->mem.alloc<unsigned long long>(1);
    HIPCHECK(hipStreamSynchronize(s));
    *out = t.release();
    return FVEM_OK;
  });
}

void fvem_transport_destroy(fvem_transport *t) { delete t; }

fvem_status fvem_locate(fvem_transport *t, int64_t n, const double *x_dev, int32_t *cell_dev, void *hip_stream) {
  if (!t || n < 0 || (n > 0 && (!x_dev || !cell_dev))) {
    g_last_error = "bad transport or arguments";
    return FVEM_ERR_INVALID;
  }
  return guard([&] {
    transport_device(t);
    locate(t->view, n, x_dev, cell_dev, static_cast<hipStream_t>(hip_stream));
    return FVEM_OK;
  });
}

fvem_status fvem_p2g(fvem_transport *t, int64_t n, const double *x_dev, const double *f_dev, int32_t m,
                     double *out_dev, void *hip_stream) {
  if (!t || n < 0 || m < 1 || m > 8 || !out_dev || (n > 0 && (!x_dev || !f_dev))) {
    g_last_error = "bad transport or arguments (1 to 8 fields per particle)";
    return FVEM_ERR_INVALID;
  }
  if (n >= (int64_t(1) << 31)) {
    g_last_error = "too many particles for int32 indices";
    return FVEM_ERR_INVALID;
  }
  TransportBusy busy(t);
  if (!busy.ok) {
    g_last_error = "transport in use by another call";
    return FVEM_ERR_BUSY;
  }
  return guard([&] {
    transport_device(t);
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (n > t->order_cap) {
      HIPCHECK(hipStreamSynchronize(s));
      t->order_mem = std::make_unique<DevMem>();
      t->order = t->order_mem->alloc<int32_t>(n);
      t->order_cap = n;
    }
    p2g(t->view, n, x_dev, f_dev, m, out_dev, t->cell_count, t->cell_start, t->chunk, t->order, s);
    return FVEM_OK;
  });
}

fvem_status fvem_buoyancy(fvem_transport *t, const double *f_dev, int32_t m, double alpha, double beta, double dt,
                          double *u_dev, void *hip_stream) {
  if (!t || m < 5 || !f_dev || !u_dev) {
    g_last_error = "bad transport or arguments (fields: u, density, temperature)";
    return FVEM_ERR_INVALID;
  }
  return guard([&] {
    transport_device(t);
    buoyancy(t->view.n_vert, f_dev, m, alpha, beta, dt, u_dev, static_cast<hipStream_t>(hip_stream));
    return FVEM_OK;
  });
}

fvem_status fvem_g2p(fvem_transport *t, int64_t n, const double *x_dev, const uint8_t *ghost_dev, double *u_dev,
                     const double *s_new_dev, const double *s_old_dev, double a_flip, void *hip_stream) {
  if (!t || n < 0 || (n > 0 && (!x_dev || !ghost_dev || !u_dev || !s_new_dev || !s_old_dev)) ||
      !(a_flip >= 0.0 && a_flip <= 1.0)) {
    g_last_error = "bad transport or arguments (a_flip in [0, 1])";
    return FVEM_ERR_INVALID;
  }
  return guard([&] {
    transport_device(t);
    g2p(t->view, n, x_dev, ghost_dev, u_dev, s_new_dev, s_old_dev, a_flip, static_cast<hipStream_t>(hip_stream));
    return FVEM_OK;
  });
}

fvem_status fvem_advect(fvem_transport *t, int64_t n, double *x_dev, const uint8_t *ghost_dev, const double *s_dev,
                        double dt, int32_t max_substeps, int32_t *substeps, void *hip_stream) {
  if (!t || n < 0 || (n > 0 && (!x_dev || !ghost_dev || !s_dev)) || !(dt >= 0.0) || max_substeps < 1) {
    g_last_error = "bad transport or arguments";
    return FVEM_ERR_INVALID;
  }
  TransportBusy busy(t);
  if (!busy.ok) {
    g_last_error = "transport in use by another call";
    return FVEM_ERR_BUSY;
  }
  return guard([&] {
    transport_device(t);
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    unsigned long long bits = 0;
    HIPCHECK(hipMemcpyAsync(t->vmax, &bits, sizeof(bits), hipMemcpyHostToDevice, s));
    grid_speed_max(t->view, n, x_dev, ghost_dev, s_dev, t->vmax, s);
    HIPCHECK(hipMemcpyAsync(&bits, t->vmax, sizeof(bits), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double vmax;
    std::memcpy(&vmax, &bits, sizeof(vmax));
    if (!std::isfinite(vmax)) throw SetupError{FVEM_ERR_NONFINITE, "non-finite grid velocity"};
    // CFL number 1 on the background spacing h = 1 / N
    const double want = std::ceil(dt * vmax * t->view.N);
    if (want > max_substeps) throw SetupError{FVEM_ERR_INVALID, "advection needs more than max_substeps substeps"};
    const int n_sub = std::max(1, static_cast<int>(want));
    advect(t->view, n, x_dev, ghost_dev, s_dev, dt, n_sub, s);
    if (substeps) *substeps = n_sub;
    return FVEM_OK;
  });
}

}  // extern "C"
