// HIP kernels for the FastVEM MG-PCG solve on CDNA4 (gfx950).
//
// Every hot kernel is HBM-bandwidth bound (SpMV-shaped, ~0.2 flop/byte);
// the only dense contraction is the coarsest-level factorisation, which runs
// on FP64 MFMA.
#include "kernels.hpp"
#include "epilogues.hpp"

#include <hip/hip_runtime.h>

namespace fvem {

// ---------------------------------------------------------------- SpMV family
//
// Vector-CSR: a group of G lanes owns one row; lanes stride over the row's
// entries (coalesced value/index loads), reduce with cross-lane shuffles and
// lane 0 applies the epilogue.  All variants read A, the gathered x and the
// per-row vectors exactly once.

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int G, typename VT, typename XT, class Epi>
__global__ __launch_bounds__(256) void spmv_kernel(int64_t n, const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const VT *__restrict__ val, const XT *__restrict__ x,
                                                   Epi epi) {
  const int64_t row = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  using AT = typename Epi::acc_t;
  AT acc = 0;
  const int64_t e = rp[row + 1];
  for (int64_t k = rp[row] + lane; k < e; k += G) acc += static_cast<AT>(val[k]) * static_cast<AT>(x[ci[k]]);
  acc = group_sum<G, AT>(acc);
  if (lane == 0) epi(row, acc);
}

static int group_for(int64_t n, int64_t nnz) {
  const double avg = n > 0 ? static_cast<double>(nnz) / n : 1.0;
  if (avg > 96) return 64;
  if (avg > 40) return 32;
  if (avg > 12) return 16;
  return 8;
}

template <typename VT, typename XT, class Epi>
static void launch_spmv(const DevCSRView<VT> &A, const XT *x, Epi epi, hipStream_t s) {
  if (A.n == 0) return;
  const int G = group_for(A.n, A.nnz);
  const int64_t rows_per_block = 256 / G;
  const dim3 grid(static_cast<unsigned>((A.n + rows_per_block - 1) / rows_per_block));
  switch (G) {
    case 64: spmv_kernel<64, VT, XT, Epi><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, A.v, x, epi); break;
    case 32: spmv_kernel<32, VT, XT, Epi><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, A.v, x, epi); break;
    case 16: spmv_kernel<16, VT, XT, Epi><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, A.v, x, epi); break;
    default: spmv_kernel<8, VT, XT, Epi><<<grid, 256, 0, s>>>(A.n, A.rp, A.ci, A.v, x, epi); break;
  }
}

template <typename T>
void spmv(const DevCSRView<T> &A, const T *x, T *y, hipStream_t s) {
  launch_spmv(A, x, EpiStore<T>{y}, s);
}
template <typename T>
void residual(const DevCSRView<T> &A, const T *x, const T *b, T *r, hipStream_t s) {
  launch_spmv(A, x, EpiResidual<T>{b, r}, s);
}
template <typename T>
void spmv_add(const DevCSRView<T> &A, const T *x, T *y, hipStream_t s) {
  launch_spmv(A, x, EpiAdd<T>{y}, s);
}
template <typename T>
void cheb_step(const DevCSRView<T> &A, const T *b, const T *dinv, const T *xin, T *d, T *xout, T ca, T cb,
               hipStream_t s) {
  launch_spmv(A, xin, EpiCheb<T>{b, dinv, xin, d, xout, ca, cb}, s);
}

void spmv_scaled(const DevCSRView<double> &A, const double *x, double *y, double alpha, hipStream_t s) {
  launch_spmv(A, x, EpiScaled{y, alpha}, s);
}

template void spmv<double>(const DevCSRView<double> &, const double *, double *, hipStream_t);
template void spmv<float>(const DevCSRView<float> &, const float *, float *, hipStream_t);
template void residual<double>(const DevCSRView<double> &, const double *, const double *, double *,
                               hipStream_t);
template void residual<float>(const DevCSRView<float> &, const float *, const float *, float *, hipStream_t);
template void spmv_add<double>(const DevCSRView<double> &, const double *, double *, hipStream_t);
template void spmv_add<float>(const DevCSRView<float> &, const float *, float *, hipStream_t);
template void cheb_step<double>(const DevCSRView<double> &, const double *, const double *, const double *,
                                double *, double *, double, double, hipStream_t);
template void cheb_step<float>(const DevCSRView<float> &, const float *, const float *, const float *,
                               float *, float *, float, float, hipStream_t);

// ---------------------------------------------------------------- vectors

template <typename T>
__global__ void cheb_first_kernel(int64_t n, const T *b, const T *dinv, T *d, T *x, T cb) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const T v = cb * dinv[i] * b[i];
    d[i] = v;
    x[i] = v;
  }
}

static dim3 vgrid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3(static_cast<unsigned>(b));
}

template <typename T>
void cheb_first(int64_t n, const T *b, const T *dinv, T *d, T *x, T cb, hipStream_t s) {
  if (n) cheb_first_kernel<<<vgrid(n), 256, 0, s>>>(n, b, dinv, d, x, cb);
}
template void cheb_first<double>(int64_t, const double *, const double *, double *, double *, double,
                                 hipStream_t);
template void cheb_first<float>(int64_t, const float *, const float *, float *, float *, float, hipStream_t);

__global__ void gather_kernel(int64_t n, const int32_t *idx, const double *x, double *y) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = idx[i] >= 0 ? x[idx[i]] : 0.0;
}

void gather(int64_t n, const int32_t *idx, const double *x, double *y, hipStream_t s) {
  if (n) gather_kernel<<<vgrid(n), 256, 0, s>>>(n, idx, x, y);
}

__global__ void lincomb_kernel(int64_t n, double alpha, const double *a, double beta, const double *b, double *y) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = b ? alpha * a[i] + beta * b[i] : alpha * a[i];
}

void lincomb(int64_t n, double alpha, const double *a, double beta, const double *b, double *y, hipStream_t s) {
  if (n) lincomb_kernel<<<vgrid(n), 256, 0, s>>>(n, alpha, a, beta, b, y);
}

__global__ void cast_scale_kernel_df(int64_t n, const double *a, float *b, double s) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b[i] = static_cast<float>(a[i] * s);
}
__global__ void cast_scale_kernel_fd(int64_t n, const float *a, double *b, double s) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b[i] = static_cast<double>(a[i]) * s;
}
void cast_scale(int64_t n, const double *a, float *b, double s, hipStream_t st) {
  if (n) cast_scale_kernel_df<<<vgrid(n), 256, 0, st>>>(n, a, b, s);
}
void cast_scale(int64_t n, const float *a, double *b, double s, hipStream_t st) {
  if (n) cast_scale_kernel_fd<<<vgrid(n), 256, 0, st>>>(n, a, b, s);
}

__global__ void axpy2_kernel(int64_t n, double alpha, const double *p, const double *q, double *x, double *r) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}
void pcg_update_xr(int64_t n, double alpha, const double *p, const double *q, double *x, double *r,
                   hipStream_t s) {
  if (n) axpy2_kernel<<<vgrid(n), 256, 0, s>>>(n, alpha, p, q, x, r);
}

__global__ void xpby_kernel(int64_t n, const double *z, double beta, double *p) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}
void pcg_update_p(int64_t n, const double *z, double beta, double *p, hipStream_t s) {
  if (n) xpby_kernel<<<vgrid(n), 256, 0, s>>>(n, z, beta, p);
}

// the same updates with alpha = num / den and beta = (num - sub) / den read
// from device scalars (outputs of the reductions), so that the host need
// not wait for them
__global__ void axpy2_dev_kernel(int64_t n, const double *num, const double *den, const double *p, const double *q,
                                 double *x, double *r) {
  const double alpha = *num / *den;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    r[i] -= alpha * q[i];
  }
}
void pcg_update_xr(int64_t n, const double *num, const double *den, const double *p, const double *q, double *x,
                   double *r, hipStream_t s) {
  if (n) axpy2_dev_kernel<<<vgrid(n), 256, 0, s>>>(n, num, den, p, q, x, r);
}

__global__ void xpby_dev_kernel(int64_t n, const double *z, const double *num, const double *sub, const double *den,
                                double *p) {
  const double beta = (*num - *sub) / *den;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}
void pcg_update_p(int64_t n, const double *z, const double *num, const double *sub, const double *den, double *p,
                  hipStream_t s) {
  if (n) xpby_dev_kernel<<<vgrid(n), 256, 0, s>>>(n, z, num, sub, den, p);
}

template <typename T>
__global__ void fill_kernel(int64_t n, T *a, T v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = v;
}
template <typename T>
void fill(int64_t n, T *a, T v, hipStream_t s) {
  if (n) fill_kernel<<<vgrid(n), 256, 0, s>>>(n, a, v);
}
template void fill<double>(int64_t, double *, double, hipStream_t);
template void fill<float>(int64_t, float *, float, hipStream_t);

// ---------------------------------------------------------------- reductions
//
// Deterministic: a fixed grid of REDUCE_BLOCKS blocks accumulates strided
// partial sums; one block adds the partials in a fixed order.  Up to four
// dot products share one pass over the vectors.

template <int NDOT>
__global__ __launch_bounds__(256) void dots_partial_kernel(int64_t n, const double *a0, const double *b0,
                                                           const double *a1, const double *b1,
                                                           const double *a2, const double *b2,
                                                           double *partial) {
  double acc[NDOT];
#pragma unroll
  for (int j = 0; j < NDOT; ++j) acc[j] = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    acc[0] += a0[i] * b0[i];
    if (NDOT > 1) acc[1] += a1[i] * b1[i];
    if (NDOT > 2) acc[2] += a2[i] * b2[i];
  }
  __shared__ double sh[NDOT][4];
#pragma unroll
  for (int j = 0; j < NDOT; ++j) {
    double v = acc[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[j][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < NDOT) {
    const int j = threadIdx.x;
    partial[j * REDUCE_BLOCKS + blockIdx.x] = ((sh[j][0] + sh[j][1]) + (sh[j][2] + sh[j][3]));
  }
}

template <int NDOT>
__global__ __launch_bounds__(256) void dots_final_kernel(const double *partial, double *out) {
  __shared__ double sh[256];
  for (int j = 0; j < NDOT; ++j) {
    double v = 0.0;
    for (int i = threadIdx.x; i < REDUCE_BLOCKS; i += 256) v += partial[j * REDUCE_BLOCKS + i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sh[0];
    __syncthreads();
  }
}

void dots(int64_t n, int ndot, const double *a0, const double *b0, const double *a1, const double *b1,
          const double *a2, const double *b2, double *partial, double *out, hipStream_t s) {
  const dim3 g(REDUCE_BLOCKS);
  switch (ndot) {
    case 1:
      dots_partial_kernel<1><<<g, 256, 0, s>>>(n, a0, b0, a1, b1, a2, b2, partial);
      dots_final_kernel<1><<<1, 256, 0, s>>>(partial, out);
      break;
    case 2:
      dots_partial_kernel<2><<<g, 256, 0, s>>>(n, a0, b0, a1, b1, a2, b2, partial);
      dots_final_kernel<2><<<1, 256, 0, s>>>(partial, out);
      break;
    default:
      dots_partial_kernel<3><<<g, 256, 0, s>>>(n, a0, b0, a1, b1, a2, b2, partial);
      dots_final_kernel<3><<<1, 256, 0, s>>>(partial, out);
      break;
  }
}

// Zero mean per pure-Neumann component (COMP_CHUNK components per pass).
// Per-component sums and counts of one block's contiguous chunk: every
// thread accumulates its strided elements into its own LDS slot per
// component, then the slots are combined by a fixed-order tree, so the
// result is independent of scheduling.  A thread keeps the slot of its
// current component in registers while consecutive elements stay in that
// component (the level order is spatial, so runs are long) and reads its
// elements four strides ahead; the additions into each slot are the same
// sequence as element-by-element LDS updates.  The slots take 4 KiB of LDS
// per component of the pass, so a one-component domain does not limit the
// blocks per CU.
constexpr int COMP_CHUNK = 16;

__global__ __launch_bounds__(256) void comp_partial_kernel(int64_t n, const double *v, const int32_t *comp,
                                                           int c0, int nc, double *partial) {
  extern __shared__ double slots[];   // nc sums, then nc counts, 256 per component
  double *s_sum = slots, *s_cnt = slots + 256 * nc;
  const int t = threadIdx.x;
  for (int j = 0; j < nc; ++j) {
    s_sum[256 * j + t] = 0.0;
    s_cnt[256 * j + t] = 0.0;
  }
  const int64_t per_block = (n + REDUCE_BLOCKS - 1) / REDUCE_BLOCKS;
  const int64_t lo = blockIdx.x * per_block;
  const int64_t hi = lo + per_block < n ? lo + per_block : n;
  int cur = -1;   // component held in (acc, cnt); -1: none
  double acc = 0.0, cnt = 0.0;
  for (int64_t i0 = lo + t; i0 < hi; i0 += 4 * 256) {
    int cc[4];
    double vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + 256 * q;
      cc[q] = -1;
      vv[q] = 0.0;
      if (i < hi) {
        const int c = comp[i] - c0;
        if (c >= 0 && c < nc) {
          cc[q] = c;
          vv[q] = v[i];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (cc[q] < 0) continue;
      if (cc[q] != cur) {
        if (cur >= 0) {
          s_sum[256 * cur + t] = acc;
          s_cnt[256 * cur + t] = cnt;
        }
        cur = cc[q];
        acc = s_sum[256 * cur + t];
        cnt = s_cnt[256 * cur + t];
      }
      acc += vv[q];
      cnt += 1.0;
    }
  }
  if (cur >= 0) {
    s_sum[256 * cur + t] = acc;
    s_cnt[256 * cur + t] = cnt;
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o)
      for (int j = 0; j < nc; ++j) {
        s_sum[256 * j + t] += s_sum[256 * j + t + o];
        s_cnt[256 * j + t] += s_cnt[256 * j + t + o];
      }
    __syncthreads();
  }
  if (t < nc) {
    partial[(2 * t) * REDUCE_BLOCKS + blockIdx.x] = s_sum[256 * t];
    partial[(2 * t + 1) * REDUCE_BLOCKS + blockIdx.x] = s_cnt[256 * t];
  }
}

__global__ void comp_final_kernel(int nc, const double *partial, double *mean) {
  const int j = blockIdx.x;
  __shared__ double sh[2][256];
  double s = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < REDUCE_BLOCKS; i += 256) {
    s += partial[(2 * j) * REDUCE_BLOCKS + i];
    c += partial[(2 * j + 1) * REDUCE_BLOCKS + i];
  }
  sh[0][threadIdx.x] = s;
  sh[1][threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[j] = sh[1][0] > 0 ? sh[0][0] / sh[1][0] : 0.0;
}

__global__ void comp_sub_kernel(int64_t n, double *v, const int32_t *comp, int c0, int nc, const double *mean) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = comp[i] - c0;
    if (c >= 0 && c < nc) v[i] -= mean[c];
  }
}

void project_components(int64_t n, double *v, const int32_t *comp, int n_comp, double *partial, double *mean,
                        hipStream_t s) {
  for (int c0 = 0; c0 < n_comp; c0 += COMP_CHUNK) {
    const int nc = n_comp - c0 < COMP_CHUNK ? n_comp - c0 : COMP_CHUNK;
    comp_partial_kernel<<<REDUCE_BLOCKS, 256, 2 * 256 * nc * sizeof(double), s>>>(n, v, comp, c0, nc, partial);
    comp_final_kernel<<<nc, 256, 0, s>>>(nc, partial, mean);
    comp_sub_kernel<<<vgrid(n), 256, 0, s>>>(n, v, comp, c0, nc, mean);
  }
}

// ---------------------------------------------------------------- Galerkin product (setup)
//
// One workgroup per coarse cell.  For each child in increasing order: K_f
// and the dense P_f (rows of the child's DOFs, columns E's local DOFs) are
// staged in LDS, T = K_f P_f is formed, and every thread adds its own
// entries of P_f^T T to K_E in global memory, so the result does not depend
// on scheduling.  Cells whose staging exceeds the LDS buffer use a slice of
// a global scratch buffer instead.

__global__ __launch_bounds__(256) void galerkin_kernel(int64_t c0, const int64_t *fptr, const int32_t *fdof,
                                                       const int64_t *kfoff, const double *kf, const int64_t *prp,
                                                       const int32_t *pci, const double *pv, const int64_t *cptr,
                                                       const int32_t *cdof, const int64_t *chptr,
                                                       const int64_t *child, const int64_t *ooff, double *out,
                                                       const int64_t *soff, double *scratch, int *bad) {
  extern __shared__ double lds[];
  const int64_t E = c0 + blockIdx.x;
  const int t = threadIdx.x;
  const int m = static_cast<int>(cptr[E + 1] - cptr[E]);
  const int32_t *cd = cdof + cptr[E];
  double *base = soff[E] >= 0 ? scratch + soff[E] : lds;
  double *KE = out + ooff[E];
  for (int64_t q = chptr[E]; q < chptr[E + 1]; ++q) {
    const int64_t f = child[q];
    const int nf = static_cast<int>(fptr[f + 1] - fptr[f]);
    const int32_t *fd = fdof + fptr[f];
    double *Kf = base, *Pf = base + nf * nf, *T = Pf + nf * m;
    const double *kblk = kf + kfoff[f];
    for (int i = t; i < nf * nf; i += 256) Kf[i] = kblk[i];
    for (int i = t; i < nf * m; i += 256) Pf[i] = 0.0;
    __syncthreads();
    for (int a = t; a < nf; a += 256) {
      const int32_t row = fd[a];
      if (row < 0) continue;
      for (int64_t k = prp[row]; k < prp[row + 1]; ++k) {
        const int32_t J = pci[k];
        int b = 0;
        while (b < m && cd[b] != J) ++b;
        if (b == m) atomicMin(bad, row);
        else Pf[a * m + b] = pv[k];
      }
    }
    __syncthreads();
    for (int i = t; i < nf * m; i += 256) {
      const int a = i / m, j = i - a * m;
      double acc = 0.0;
      for (int b = 0; b < nf; ++b) acc += Kf[a * nf + b] * Pf[b * m + j];
      T[i] = acc;
    }
    __syncthreads();
    for (int i = t; i < m * m; i += 256) {
      const int r = i / m, j = i - r * m;
      double acc = 0.0;
      for (int a = 0; a < nf; ++a) acc += Pf[a * m + r] * T[a * m + j];
      KE[i] += acc;
    }
    __syncthreads();
  }
}

void galerkin(int64_t c0, int64_t ncells, const int64_t *fptr, const int32_t *fdof, const int64_t *kfoff,
              const double *kf, const int64_t *prp, const int32_t *pci, const double *pv, const int64_t *cptr,
              const int32_t *cdof, const int64_t *chptr, const int64_t *child, const int64_t *ooff, double *out,
              const int64_t *soff, double *scratch, int *bad, hipStream_t s) {
  if (ncells <= 0) return;
  galerkin_kernel<<<static_cast<unsigned>(ncells), 256, GALERKIN_LDS_DOUBLES * sizeof(double), s>>>(
      c0, fptr, fdof, kfoff, kf, prp, pci, pv, cptr, cdof, chptr, child, ooff, out, soff, scratch, bad);
}

// ---------------------------------------------------------------- dense FP64 (coarsest level)
//
// Symmetric positive semi-definite factorisation A = L L^T, right-looking in
// column blocks of NB: factor the diagonal block in LDS (a pivot below
// rcond * a_jj of the original matrix zeroes its column), solve the panel
// below it, update the trailing matrix with an FP64 MFMA GEMM.  Matrices are
// column-major with leading dimension ld.

constexpr int NB = 64;

__global__ __launch_bounds__(256) void potrf_diag_kernel(double *A, int64_t ld, int64_t k0, int nb,
                                                         const double *diag0, double rcond, int *flag) {
  __shared__ double L[NB][NB + 1];
  for (int t = threadIdx.x; t < nb * nb; t += 256) {
    const int i = t % nb, j = t / nb;
    L[i][j] = A[(k0 + i) + (k0 + j) * ld];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double d = L[j][j];
    const double thr = rcond * diag0[k0 + j];
    __syncthreads();
    const bool zero = !(d > thr);
    if (threadIdx.x == 0 && d < -1e-6 * diag0[k0 + j]) atomicOr(flag, 1);
    const double piv = zero ? 0.0 : sqrt(d);
    if (threadIdx.x == 0) L[j][j] = piv;
    for (int i = j + 1 + threadIdx.x; i < nb; i += 256) L[i][j] = zero ? 0.0 : L[i][j] / piv;
    __syncthreads();
    // trailing update inside the block (lower triangle)
    for (int t = threadIdx.x; t < nb * nb; t += 256) {
      const int i = t % nb, c = t / nb;
      if (c > j && i >= c) L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nb * nb; t += 256) {
    const int i = t % nb, j = t / nb;
    A[(k0 + i) + (k0 + j) * ld] = (i >= j) ? L[i][j] : 0.0;
  }
}

// Rows below the diagonal block: L21 = A21 L11^-T (row-parallel forward substitution).
__global__ __launch_bounds__(256) void trsm_panel_kernel(double *A, int64_t ld, int64_t n, int64_t k0, int nb) {
  __shared__ double L[NB][NB + 1];
  for (int t = threadIdx.x; t < nb * nb; t += 256) {
    const int i = t % nb, j = t / nb;
    L[i][j] = A[(k0 + i) + (k0 + j) * ld];
  }
  __syncthreads();
  const int64_t row = k0 + nb + blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (row >= n) return;
  double x[NB];
  for (int j = 0; j < nb; ++j) {
    double s = A[row + (k0 + j) * ld];
    for (int t = 0; t < j; ++t) s -= x[t] * L[j][t];
    x[j] = (L[j][j] != 0.0) ? s / L[j][j] : 0.0;
  }
  for (int j = 0; j < nb; ++j) A[row + (k0 + j) * ld] = x[j];
}

// C (+)= alpha op(A) op(B) on FP64 MFMA (v_mfma_f64_16x16x4f64), with
// op(A)(i,k) = A[i*sai + k*sak], op(B)(k,j) = B[k*sbk + j*sbj] and C
// column-major (ldc).  A workgroup of 4 wavefronts computes a 64 x 64 block
// of C; wavefront w owns the 32 x 32 quarter (w & 1, w >> 1) as 2 x 2 MFMA
// tiles.  K is walked in chunks of 16: both operands' 64 x 16 panels are
// staged in LDS, k-major, so a block reads each global element once per
// chunk (8 flop per byte from L2 instead of 2 with per-tile loads).  With
// lower_only, blocks wholly above the diagonal are skipped; the blocks that
// straddle it are computed whole.
typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int GEMM_B = 64, GEMM_K = 16;
// LDS row pitch: 80 doubles puts consecutive k rows 32 banks apart, so the
// two k rows read by each half-wavefront fall on distinct banks
constexpr int GEMM_PITCH = GEMM_B + 16;

__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                       const double *A, int64_t sai, int64_t sak,
                                                       const double *B, int64_t sbk, int64_t sbj, double beta,
                                                       double *C, int64_t ldc, int lower_only) {
  __shared__ double As[GEMM_K * GEMM_PITCH];
  __shared__ double Bs[GEMM_K * GEMM_PITCH];
  const int64_t ib = static_cast<int64_t>(blockIdx.x) * GEMM_B;
  const int64_t jb = static_cast<int64_t>(blockIdx.y) * GEMM_B;
  if (lower_only && ib + GEMM_B - 1 < jb) return;   // whole workgroup
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int r = lane & 15;   // row of A / column of B inside a 16 x 16 tile
  const int kk = lane >> 4;  // k inside a 4-step
  // panel loads run along whichever index is contiguous in memory
  const bool a_i_fast = sai == 1, b_j_fast = sbj == 1;
  double4_t acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[m][n] = double4_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t kb = 0; kb < K; kb += GEMM_K) {
    double va[4], vb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ia = a_i_fast ? (e & 63) : (e >> 4), ka = a_i_fast ? (e >> 6) : (e & 15);
      const int jb_ = b_j_fast ? (e & 63) : (e >> 4), kb_ = b_j_fast ? (e >> 6) : (e & 15);
      const int64_t gi = ib + ia, gka = kb + ka, gj = jb + jb_, gkb = kb + kb_;
      va[q] = (gi < M && gka < K) ? A[gi * sai + gka * sak] : 0.0;
      vb[q] = (gj < N && gkb < K) ? B[gkb * sbk + gj * sbj] : 0.0;
    }
    __syncthreads();   // the previous chunk's reads of As and Bs are done
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ia = a_i_fast ? (e & 63) : (e >> 4), ka = a_i_fast ? (e >> 6) : (e & 15);
      const int jb_ = b_j_fast ? (e & 63) : (e >> 4), kb_ = b_j_fast ? (e >> 6) : (e & 15);
      As[ka * GEMM_PITCH + ia] = va[q];
      Bs[kb_ * GEMM_PITCH + jb_] = vb[q];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GEMM_K; ks += 4) {
      double a[2], b[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) a[m] = As[(ks + kk) * GEMM_PITCH + wr + 16 * m + r];
#pragma unroll
      for (int n = 0; n < 2; ++n) b[n] = Bs[(ks + kk) * GEMM_PITCH + wc + 16 * n + r];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[n], acc[m][n], 0, 0, 0);
    }
  }
  // D layout (measured on gfx950): register q of a lane holds row
  // (lane / 16) + 4 q, column lane % 16 of its 16 x 16 tile
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = ib + wr + 16 * m + (lane >> 4) + 4 * q;
        const int64_t j = jb + wc + 16 * n + (lane & 15);
        if (i < M && j < N) {
          double *c = C + i + j * ldc;
          *c = alpha * acc[m][n][q] + (beta == 0.0 ? 0.0 : beta * *c);
        }
      }
}

void gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t sai, int64_t sak,
              const double *B, int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc, bool lower_only,
              hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const dim3 g(static_cast<unsigned>((M + GEMM_B - 1) / GEMM_B), static_cast<unsigned>((N + GEMM_B - 1) / GEMM_B));
  gemm_f64_kernel<<<g, 256, 0, s>>>(M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, ldc, lower_only ? 1 : 0);
}

void potrf_semidefinite(double *A, int64_t n, const double *diag0, double rcond, int *flag, hipStream_t s) {
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int nb = static_cast<int>(n - k0 < NB ? n - k0 : NB);
    potrf_diag_kernel<<<1, 256, 0, s>>>(A, n, k0, nb, diag0, rcond, flag);
    const int64_t rest = n - k0 - nb;
    if (rest <= 0) break;
    trsm_panel_kernel<<<static_cast<unsigned>((rest + 255) / 256), 256, 0, s>>>(A, n, n, k0, nb);
    // A22 -= L21 L21^T (lower triangle)
    const double *L21 = A + (k0 + nb) + k0 * n;
    double *A22 = A + (k0 + nb) + (k0 + nb) * n;
    gemm_f64(rest, rest, nb, -1.0, L21, 1, n, L21, n, 1, 1.0, A22, n, true, s);
  }
}

// X = L^+ (lower triangular, zero rows for zero pivots): block forward
// substitution on the identity.  Block row i: T = E_i - L[i,0:i] X[0:i,0:i],
// then X[i,0:i+1] = L_ii^+ T, column-parallel inside the block.
__global__ __launch_bounds__(256) void trinv_block_kernel(const double *L, double *X, int64_t n, int64_t i0,
                                                          int nb) {
  __shared__ double Lb[NB][NB + 1];
  for (int t = threadIdx.x; t < nb * nb; t += 256) {
    const int a = t % nb, b = t / nb;
    Lb[a][b] = L[(i0 + a) + (i0 + b) * n];
  }
  __syncthreads();
  const int64_t col = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (col >= i0 + nb) return;
  double x[NB];
  for (int a = 0; a < nb; ++a) {
    double s = X[(i0 + a) + col * n];          // holds T (minus the identity)
    if (col == i0 + a) s += 1.0;
    for (int t = 0; t < a; ++t) s -= Lb[a][t] * x[t];
    x[a] = (Lb[a][a] != 0.0) ? s / Lb[a][a] : 0.0;
  }
  for (int a = 0; a < nb; ++a) X[(i0 + a) + col * n] = x[a];
}

void trinv_semidefinite(const double *L, double *X, int64_t n, hipStream_t s) {
  (void)hipMemsetAsync(X, 0, sizeof(double) * n * n, s);
  for (int64_t i0 = 0; i0 < n; i0 += NB) {
    const int nb = static_cast<int>(n - i0 < NB ? n - i0 : NB);
    if (i0 > 0) {
      // X[i0:i0+nb, 0:i0] = -L[i0:i0+nb, 0:i0] X[0:i0, 0:i0]
      gemm_f64(nb, i0, i0, -1.0, L + i0, 1, n, X, 1, n, 0.0, X + i0, n, false, s);
    }
    trinv_block_kernel<<<static_cast<unsigned>((i0 + nb + 255) / 256), 256, 0, s>>>(L, X, n, i0, nb);
  }
}

// Symmetric dense y = G x (FP64), one wave per row block of 4 rows? keep simple:
// one 256-thread block per row, coalesced along the row of the column-major
// symmetric matrix (row i of G = column i).
__global__ __launch_bounds__(256) void symv_kernel(int64_t n, const double *G, const double *x, double *y) {
  const int64_t i = blockIdx.x;
  const double *col = G + i * n;
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) acc += col[k] * x[k];
  __shared__ double sh[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) y[i] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

void symv(int64_t n, const double *G, const double *x, double *y, hipStream_t s) {
  if (n) symv_kernel<<<static_cast<unsigned>(n), 256, 0, s>>>(n, G, x, y);
}

__global__ void dense_from_csr_kernel(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                                      double *D) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) D[i + static_cast<int64_t>(ci[k]) * n] = v[k];
}

void dense_from_csr(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double *D, hipStream_t s) {
  (void)hipMemsetAsync(D, 0, sizeof(double) * n * n, s);
  if (n) dense_from_csr_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(n, rp, ci, v, D);
}

__global__ void add_diagonal_kernel(int64_t n, double *D, const double *v) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) D[i + i * n] += v[i];
}

void add_diagonal(int64_t n, double *D, const double *v, hipStream_t s) {
  if (n) add_diagonal_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(n, D, v);
}

__global__ void cast_f64_f32_kernel(int64_t n, const double *a, float *b) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b[i] = static_cast<float>(a[i]);
}
void cast_f64_f32(int64_t n, const double *a, float *b, hipStream_t s) {
  if (n) cast_f64_f32_kernel<<<vgrid(n), 256, 0, s>>>(n, a, b);
}

}  // namespace fvem
