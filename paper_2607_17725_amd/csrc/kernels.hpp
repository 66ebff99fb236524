// Kernel launchers of the FastVEM solver (implemented in kernels.hip).
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace fvem {

constexpr int REDUCE_BLOCKS = 1024;
constexpr int MAX_COMP = 64;

template <typename T>
struct DevCSRView {
  int64_t n = 0, m = 0, nnz = 0;
  const int64_t *rp = nullptr;
  const int32_t *ci = nullptr;
  const T *v = nullptr;
};

// Lattice stencil rows of a level operator (see HostLattice in
// setup_host.hpp): one workgroup per tile listed in tiles; x of the tile
// plus a 2-point halo is staged in LDS by class, and each wavefront applies
// its class's table to the slots flagged in the tile's mask.
template <typename T>
struct StencilView {
  int64_t ntiles = 0;
  const int32_t *tiles = nullptr;      // tile ids, launch order
  const uint64_t *mask = nullptr;      // 8 words per launched tile
  const int32_t *tile_base = nullptr;  // tn^3 slot bases (-1: no slots)
  int32_t tn = 0, lat_n = 0;
  const int32_t *len = nullptr;        // 8 entry counts
  const int32_t *off = nullptr;        // 8 x 128 LDS offsets
  const T *val = nullptr;              // 8 x 128 values
  const T *dinv = nullptr;             // 8: 1 / (diagonal of each class's stencil)
  bool standard = false;               // every class has the full order-2 support (unrolled kernel)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // recorded around the stencil launch when set
};

// Sliced ELLPACK with 64-row slices (one wavefront lane per row).  Slice s
// holds rows [64 s, 64 s + 64); entry j of lane r sits at o = 256 (j / 4) +
// 4 r + j % 4 from the slice's start, for j < sl[s] (the slice's longest row
// rounded up to 4).  Columns: ci[cp[s] + o], or for coded slices (bt[s] >= 0)
// btab[bt[s] + (c16[cp[s] + o] >> 10)] + (c16[cp[s] + o] & 1023).  Values:
// when vp[s] >= 0 at v[vp[s] + o]; when vp[s] < 0 every row of the slice
// takes them from its template, tv[tid[row] * tw + j].  Shorter rows are
// padded with value 0 and a valid column.
template <typename T>
struct DevSELLView {
  int64_t n = 0, m = 0, nslices = 0;
  const int32_t *sl = nullptr;
  const int64_t *cp = nullptr;     // per slice: column offset in ci (bt < 0) or c16 (bt >= 0)
  const int32_t *ci = nullptr;
  const int64_t *bt = nullptr;     // per slice: block-table offset in btab, or -1
  const uint16_t *c16 = nullptr;   // 16-bit column codes (block index << 10 | offset)
  const int32_t *btab = nullptr;   // block starts, 64 per coded slice
  const int64_t *vp = nullptr;
  const T *v = nullptr;
  const int32_t *tid = nullptr;
  const T *tv = nullptr;
  int32_t tw = 0;
  bool split = false;   // several lanes per row (small levels)
  const int32_t *rowmap = nullptr;   // stored row r is output row rowmap[r] (null: r)
  StencilView<T> st;    // lattice stencil rows applied before the sliced rows (ntiles 0: none)
};

// SpMV family on the sliced layout (level operators; fused epilogues)
template <typename T> void spmv(const DevSELLView<T> &A, const T *x, T *y, hipStream_t s);
template <typename T> void residual(const DevSELLView<T> &A, const T *x, const T *b, T *r, hipStream_t s);
template <typename T>
void cheb_step(const DevSELLView<T> &A, const T *b, const T *dinv, const T *xin, T *d, T *xout, T ca, T cb,
               hipStream_t s);
template <typename T> void spmv_add(const DevSELLView<T> &A, const T *x, T *y, hipStream_t s);

// SpMV family (vector CSR with fused epilogues; transfers and divergence)
template <typename T> void spmv(const DevCSRView<T> &A, const T *x, T *y, hipStream_t s);
template <typename T> void residual(const DevCSRView<T> &A, const T *x, const T *b, T *r, hipStream_t s);
template <typename T> void spmv_add(const DevCSRView<T> &A, const T *x, T *y, hipStream_t s);
void spmv_scaled(const DevCSRView<double> &A, const double *x, double *y, double alpha, hipStream_t s);  // y = alpha A x
template <typename T>
void cheb_step(const DevCSRView<T> &A, const T *b, const T *dinv, const T *xin, T *d, T *xout, T ca, T cb,
               hipStream_t s);
template <typename T> void cheb_first(int64_t n, const T *b, const T *dinv, T *d, T *x, T cb, hipStream_t s);

// vectors
void gather(int64_t n, const int32_t *idx, const double *x, double *y, hipStream_t s);   // y[i] = x[idx[i]] (0 where idx[i] < 0)
// y = alpha a + beta b (b may be null: y = alpha a); y may alias a or b
void lincomb(int64_t n, double alpha, const double *a, double beta, const double *b, double *y, hipStream_t s);
void cast_scale(int64_t n, const double *a, float *b, double s, hipStream_t st);
void cast_scale(int64_t n, const float *a, double *b, double s, hipStream_t st);
void cast_f64_f32(int64_t n, const double *a, float *b, hipStream_t s);
void pcg_update_xr(int64_t n, double alpha, const double *p, const double *q, double *x, double *r,
                   hipStream_t s);
void pcg_update_p(int64_t n, const double *z, double beta, double *p, hipStream_t s);
// x += a p, r -= a q with a = *num / *den (device scalars)
void pcg_update_xr(int64_t n, const double *num, const double *den, const double *p, const double *q, double *x,
                   double *r, hipStream_t s);
// p = z + b p with b = (*num - *sub) / *den (device scalars)
void pcg_update_p(int64_t n, const double *z, const double *num, const double *sub, const double *den, double *p,
                  hipStream_t s);
template <typename T> void fill(int64_t n, T *a, T v, hipStream_t s);

// deterministic reductions: out[j] = a_j . b_j for j < ndot (ndot <= 3);
// partial needs 3 * REDUCE_BLOCKS doubles
void dots(int64_t n, int ndot, const double *a0, const double *b0, const double *a1, const double *b1,
          const double *a2, const double *b2, double *partial, double *out, hipStream_t s);
// v -= mean over each pure-Neumann component; partial needs 2 * MAX_COMP * REDUCE_BLOCKS doubles
void project_components(int64_t n, double *v, const int32_t *comp, int n_comp, double *partial, double *mean,
                        hipStream_t s);

// Element-wise Galerkin product on the device (setup, Sec. 4):
//   K_E = sum over fine cells f with parent E of P_f^T K_f P_f
// for coarse cells E in [c0, c0 + ncells).  P_f is the dense block of P's
// rows of f's DOFs on E's local DOFs (built per child in LDS or, where
// soff[E] >= 0, in the global scratch at that offset).  fptr/fdof and
// cptr/cdof are the fine and coarse cell DOF lists (-1: eliminated),
// kfoff/kf the fine blocks (row-major n_f x n_f), chptr/child the children
// of each coarse cell in increasing order, ooff/out the coarse blocks
// (row-major m_E x m_E, zero on entry).  A P row that references a DOF
// outside E sets *bad to the smallest such fine row.
constexpr int GALERKIN_LDS_DOUBLES = 8192;
void galerkin(int64_t c0, int64_t ncells, const int64_t *fptr, const int32_t *fdof, const int64_t *kfoff,
              const double *kf, const int64_t *prp, const int32_t *pci, const double *pv, const int64_t *cptr,
              const int32_t *cdof, const int64_t *chptr, const int64_t *child, const int64_t *ooff, double *out,
              const int64_t *soff, double *scratch, int *bad, hipStream_t s);

// dense FP64 (coarsest level), column-major
void gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t sai, int64_t sak,
              const double *B, int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc, bool lower_only,
              hipStream_t s);
void potrf_semidefinite(double *A, int64_t n, const double *diag0, double rcond, int *flag, hipStream_t s);
void trinv_semidefinite(const double *L, double *X, int64_t n, hipStream_t s);
void symv(int64_t n, const double *G, const double *x, double *y, hipStream_t s);
void add_diagonal(int64_t n, double *D, const double *v, hipStream_t s);   // D_ii += v_i
void dense_from_csr(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double *D, hipStream_t s);

}  // namespace fvem
