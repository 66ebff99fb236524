// Sliced-ELLPACK SpMV family of the level operators (a4 SpMV, a5 Chebyshev
// step, a6 residual) on CDNA4 (gfx950).  Layout and value templates are
// built on the host by to_sell (setup_host.cpp).
#include <hip/hip_runtime.h>

#include "epilogues.hpp"
#include "kernels.hpp"
#include "setup_host.hpp"

namespace fvem {

// Sliced ELLPACK: one wavefront per 64-row slice, one lane per row, so the
// value and column loads of a step are contiguous reads per wavefront.  Rows
// inside each window of the level order are sorted by length at setup, so a
// slice's rows have (nearly) equal length and padding is a few percent.  The matrix is streamed once per
// launch with non-temporal loads, leaving the caches to the gathered x.
// Workgroups are dispatched round-robin over the 8 XCDs; remapping the
// workgroup id gives each XCD a contiguous range of slices, so x entries
// shared by neighbouring slices are reused in that XCD's L2.

__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7;
  const int64_t xcd = b & 7, idx = b >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// 4-wide vectors for the interleaved groups of 4 entries
typedef int32_t int4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef double double2v __attribute__((ext_vector_type(2)));

template <typename T> struct Quad;
template <> struct Quad<float> {
  __device__ static void load_nt(const float *p, float v[4]) {
    const float4v q = __builtin_nontemporal_load(reinterpret_cast<const float4v *>(p));
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ static void load(const float *p, float v[4]) {
    const float4v q = *reinterpret_cast<const float4v *>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};
template <> struct Quad<double> {
  __device__ static void load_nt(const double *p, double v[4]) {
    const double2v a = __builtin_nontemporal_load(reinterpret_cast<const double2v *>(p));
    const double2v b = __builtin_nontemporal_load(reinterpret_cast<const double2v *>(p + 2));
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  __device__ static void load(const double *p, double v[4]) {
    const double2v a = *reinterpret_cast<const double2v *>(p);
    const double2v b = *reinterpret_cast<const double2v *>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};

// Entry j of lane r of a slice sits at 256 (j / 4) + 4 r + j % 4 from the
// slice start: each group of 4 entries is one 16-byte load per lane and one
// contiguous 1 KiB read per wavefront.  SELL_GROUPS groups are in flight per
// step.
constexpr int SELL_GROUPS = 4;
// 8 slices (wavefronts) per workgroup: with the level order's spatially
// ordered slices this is one 4x4x4-cell tile of k = 2 DOFs, whose gathers
// of x share the CU's L1.
constexpr int SELL_WAVES = 8;

typedef uint16_t ushort4v __attribute__((ext_vector_type(4)));

// Column sources of a lane's group g (4 entries).  Plain: int32 columns.
// Coded: 16-bit codes (block << 10 | offset); the slice's 64 block starts
// sit one per lane of the wavefront and are fetched with a cross-lane read.
struct ColsPlain {
  const int32_t *cp;
  __device__ int4v operator()(int g) const {
    return __builtin_nontemporal_load(reinterpret_cast<const int4v *>(cp + 256 * static_cast<int64_t>(g)));
  }
};
struct ColsCoded {
  const uint16_t *cq;
  int32_t tab;   // this lane's block start
  __device__ int4v operator()(int g) const {
    const ushort4v q = __builtin_nontemporal_load(reinterpret_cast<const ushort4v *>(cq + 256 * static_cast<int64_t>(g)));
    int4v c;
    c.x = __shfl(tab, q.x >> 10) + (q.x & 1023);
    c.y = __shfl(tab, q.y >> 10) + (q.y & 1023);
    c.z = __shfl(tab, q.z >> 10) + (q.z & 1023);
    c.w = __shfl(tab, q.w >> 10) + (q.w & 1023);
    return c;
  }
};
// Value sources: stored with the slice (streamed) or a template row (cached).
template <typename VT> struct ValsStored {
  const VT *vq;
  __device__ void operator()(int g, VT v[4]) const { Quad<VT>::load_nt(vq + 256 * static_cast<int64_t>(g), v); }
};
template <typename VT> struct ValsTemplate {
  const VT *tq;
  __device__ void operator()(int g, VT v[4]) const { Quad<VT>::load(tq + 4 * g, v); }
};

// sum over a row's groups, SELL_GROUPS of them in flight
template <typename AT, typename VT, typename XT, class Cols, class Vals>
__device__ __forceinline__ AT row_sum(int groups, const Cols &cols, const Vals &vals, const XT *__restrict__ x) {
  AT acc = 0;
  auto fma4 = [&](const int4v c, const VT v[4]) {
    acc += static_cast<AT>(v[0]) * static_cast<AT>(x[c.x]);
    acc += static_cast<AT>(v[1]) * static_cast<AT>(x[c.y]);
    acc += static_cast<AT>(v[2]) * static_cast<AT>(x[c.z]);
    acc += static_cast<AT>(v[3]) * static_cast<AT>(x[c.w]);
  };
  int g = 0;
  for (; g + SELL_GROUPS <= groups; g += SELL_GROUPS) {
    int4v c[SELL_GROUPS];
    VT v[SELL_GROUPS][4];
#pragma unroll
    for (int u = 0; u < SELL_GROUPS; ++u) {
      c[u] = cols(g + u);
      vals(g + u, v[u]);
    }
#pragma unroll
    for (int u = 0; u < SELL_GROUPS; ++u) fma4(c[u], v[u]);
  }
  for (; g < groups; ++g) {
    VT v0[4];
    vals(g, v0);
    fma4(cols(g), v0);
  }
  return acc;
}

template <typename VT, typename XT, class Epi>
__device__ __forceinline__ void sell_block(
    int64_t blk, int64_t n, int64_t nslices, const int32_t *__restrict__ sl, const int64_t *__restrict__ cpo,
    const int32_t *__restrict__ ci, const int64_t *__restrict__ bt, const uint16_t *__restrict__ c16,
    const int32_t *__restrict__ btab, const int64_t *__restrict__ vp, const VT *__restrict__ val,
    const int32_t *__restrict__ tid, const VT *__restrict__ tv, int32_t tw, const int32_t *__restrict__ rowmap,
    const XT *__restrict__ x, const Epi &epi) {
  const int64_t slice = blk * SELL_WAVES + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slice >= nslices) return;   // whole wavefronts only: every lane below takes part in the cross-lane reads
  using AT = typename Epi::acc_t;
  const int groups = sl[slice] >> 2;
  const int64_t co = cpo[slice] + 4 * lane;
  const int64_t bto = bt[slice];
  const int64_t vb = vp[slice];
  AT acc;
  if (bto >= 0) {
    const ColsCoded cols{c16 + co, btab[bto + lane]};
    if (vb >= 0) acc = row_sum<AT, VT>(groups, cols, ValsStored<VT>{val + vb + 4 * lane}, x);
    else acc = row_sum<AT, VT>(groups, cols, ValsTemplate<VT>{tv + static_cast<int64_t>(tid[slice * 64 + lane]) * tw}, x);
  } else {
    const ColsPlain cols{ci + co};
    if (vb >= 0) acc = row_sum<AT, VT>(groups, cols, ValsStored<VT>{val + vb + 4 * lane}, x);
    else acc = row_sum<AT, VT>(groups, cols, ValsTemplate<VT>{tv + static_cast<int64_t>(tid[slice * 64 + lane]) * tw}, x);
  }
  const int64_t row = slice * 64 + lane;
  if (row < n) epi(rowmap ? static_cast<int64_t>(rowmap[row]) : row, acc);
}

template <typename VT, typename XT, class Epi>
__global__ __launch_bounds__(64 * SELL_WAVES) void sell_kernel(
    int64_t n, int64_t nslices, const int32_t *__restrict__ sl, const int64_t *__restrict__ cpo,
    const int32_t *__restrict__ ci, const int64_t *__restrict__ bt, const uint16_t *__restrict__ c16,
    const int32_t *__restrict__ btab, const int64_t *__restrict__ vp, const VT *__restrict__ val,
    const int32_t *__restrict__ tid, const VT *__restrict__ tv, int32_t tw, const int32_t *__restrict__ rowmap,
    const XT *__restrict__ x, Epi epi) {
  sell_block<VT, XT, Epi>(xcd_contiguous(blockIdx.x, gridDim.x), n, nslices, sl, cpo, ci, bt, c16, btab, vp, val,
                          tid, tv, tw, rowmap, x, epi);
}

// Small levels (a few thousand slices) cannot fill 256 CUs with one
// wavefront per slice, and each wavefront would walk its rows' 60-300
// entries serially.  There, SPLIT lanes share a row: lane k of a row takes
// the row's groups k, k + SPLIT, ... in order, and the lanes' sums are
// combined by a fixed butterfly, so the result is still deterministic.
constexpr int SELL_SPLIT = 16;

template <typename VT, typename XT, class Epi>
__global__ __launch_bounds__(256) void sell_split_kernel(
    int64_t n, const int32_t *__restrict__ sl, const int64_t *__restrict__ cpo, const int32_t *__restrict__ ci,
    const int64_t *__restrict__ bt, const uint16_t *__restrict__ c16, const int32_t *__restrict__ btab,
    const int64_t *__restrict__ vp, const VT *__restrict__ val, const int32_t *__restrict__ tid,
    const VT *__restrict__ tv, int32_t tw, const int32_t *__restrict__ rowmap, const XT *__restrict__ x, Epi epi) {
  const int64_t row = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / SELL_SPLIT;
  const int k = threadIdx.x % SELL_SPLIT;
  if (row >= n) return;
  using AT = typename Epi::acc_t;
  const int64_t slice = row >> 6;
  const int q = static_cast<int>(row & 63);
  const int groups = sl[slice] >> 2;
  const int64_t co = cpo[slice] + 4 * q;
  const int64_t bto = bt[slice];
  const int64_t vb = vp[slice];
  const VT *vq = vb >= 0 ? val + vb + 4 * q : nullptr;
  const VT *tq = vb >= 0 ? nullptr : tv + static_cast<int64_t>(tid[row]) * tw;
  AT acc = 0;
  for (int g = k; g < groups; g += SELL_SPLIT) {
    int4v c;
    if (bto >= 0) {
      // codes decoded through the slice's block table (cache resident)
      const ushort4v u = *reinterpret_cast<const ushort4v *>(c16 + co + 256 * static_cast<int64_t>(g));
      c.x = btab[bto + (u.x >> 10)] + (u.x & 1023);
      c.y = btab[bto + (u.y >> 10)] + (u.y & 1023);
      c.z = btab[bto + (u.z >> 10)] + (u.z & 1023);
      c.w = btab[bto + (u.w >> 10)] + (u.w & 1023);
    } else {
      c = *reinterpret_cast<const int4v *>(ci + co + 256 * static_cast<int64_t>(g));
    }
    VT v[4];
    if (vq) Quad<VT>::load(vq + 256 * static_cast<int64_t>(g), v);
    else Quad<VT>::load(tq + 4 * g, v);
    acc += static_cast<AT>(v[0]) * static_cast<AT>(x[c.x]);
    acc += static_cast<AT>(v[1]) * static_cast<AT>(x[c.y]);
    acc += static_cast<AT>(v[2]) * static_cast<AT>(x[c.z]);
    acc += static_cast<AT>(v[3]) * static_cast<AT>(x[c.w]);
  }
#pragma unroll
  for (int o = SELL_SPLIT / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, SELL_SPLIT);
  if (k == 0) epi(rowmap ? static_cast<int64_t>(rowmap[row]) : row, acc);
}

// Lattice stencil rows.  A tile's 8^3 points plus a 2-point halo (12^3 =
// 1728 values) are staged in LDS, split by class into 6^3 sub-grids with
// pitches of 8 per row and 68 per plane.  The class table (LDS offset,
// value) is wave-uniform, so its entries come through scalar loads; every
// row sums its entries in the table's fixed order (deterministic).
// Rows of class T = 4 ta + 2 tb + tc with the standard order-2 support:
// offsets in [-2, 2] along even coordinates and [-1, 1] along odd ones, in
// the table's order (increasing offset code).  Offsets and LDS addresses are
// compile-time constants; the values come from the table.
// Each lane sums two rows of class T, neighbours along b (sub-grid rows pj
// and pj + 1 of one tile): the lattice offsets db of the first row and
// db - 2 of the second share their x values, so each value of the union
// [-rb, rb + 2] is read from LDS once (a quarter fewer reads than one row
// per lane).  Each row still adds its entries in the table's order, so the
// sums equal those of one row per lane.  The 32 lanes of a half-wavefront
// (4 planes, 2 row pairs, 4 columns) fall on distinct banks.  hp is the
// first row's base in the lane's first tile; its tiles are TS apart in LDS.
template <int T, int NL, int TS, typename VT, typename XT, typename AT>
__device__ __forceinline__ void stencil_pairs_std(const XT *hp, const VT *val, AT acc[NL][2]) {
  constexpr int ta = T >> 2, tb = (T >> 1) & 1, tc = T & 1;
  constexpr int ra = ta ? 1 : 2, rb = tb ? 1 : 2, rc = tc ? 1 : 2;
  constexpr int nb = 2 * rb + 1, nc = 2 * rc + 1;
#pragma unroll
  for (int v = 0; v < NL; ++v) acc[v][0] = acc[v][1] = 0;
#pragma unroll
  for (int da = -ra; da <= ra; ++da)
#pragma unroll
    for (int e = -rb; e <= rb + 2; ++e)
#pragma unroll
      for (int dc = -rc; dc <= rc; ++dc) {
        const int ua = (ta + da) & 1, ub = (tb + e) & 1, uc = (tc + dc) & 1;
        const int off = (4 * ua + 2 * ub + uc) * STENCIL_SUB + ((ta + da + 2 - ua) / 2) * STENCIL_P1 +
                        ((tb + e + 2 - ub) / 2) * STENCIL_P2 + (tc + dc + 2 - uc) / 2;
        const int j0 = ((da + ra) * nb + (e + rb)) * nc + (dc + rc);       // first row, db = e
        const int j1 = ((da + ra) * nb + (e - 2 + rb)) * nc + (dc + rc);   // second row, db = e - 2
#pragma unroll
        for (int v = 0; v < NL; ++v) {
          const AT xv = static_cast<AT>(hp[v * TS + off]);
          if (e <= rb) acc[v][0] += static_cast<AT>(val[j0]) * xv;
          if (e - 2 >= -rb) acc[v][1] += static_cast<AT>(val[j1]) * xv;
        }
      }
}

// Tiles per stencil workgroup (even: a half-wavefront takes every other
// tile).  The tiles of one workgroup share its latency chain (tile ids,
// neighbour bases, the barriers) and its class tables.  Measured on the
// 128^3 plates (FP32 Chebyshev step): with one row per lane, 1, 2, 3, 4
// tiles took 0.247, 0.201, 0.190, 0.223 ms; with two rows per lane, 2, 4, 6
// tiles take 0.164, 0.169, 0.203 ms.
constexpr int STENCIL_TPW = 2;

// One workgroup of 8 wavefronts per STENCIL_TPW consecutive tiles;
// wavefront t handles the slots of class t.  Every tile's 8^3 points plus a
// 2-point halo (12^3 values) are staged in LDS, split by class into 6^3
// sub-grids; each lane then sums two rows of its class (sub-grid rows pj and
// pj + 1) per tile of its half-wavefront.
template <typename VT, typename XT, class Epi>
__global__ __launch_bounds__(512) void stencil_kernel(StencilView<VT> st, const XT *__restrict__ x, Epi epi) {
  constexpr int NT = STENCIL_TPW, NL = NT / 2, TILE = 8 * STENCIL_SUB;
  __shared__ XT halo[NT * TILE];
  __shared__ int32_t nbase[NT][27];
  const int64_t b0 = NT * xcd_contiguous(blockIdx.x, gridDim.x);
  const int nt = static_cast<int>(min(static_cast<int64_t>(NT), st.ntiles - b0));
  const int tn = st.tn, N = st.lat_n;
  if (threadIdx.x < 32 * NT) {
    const int u = threadIdx.x >> 5, j = threadIdx.x & 31;
    if (j < 27 && u < nt) {
      const int32_t tile = st.tiles[b0 + u];
      const int Ta = tile / (tn * tn), Tb = (tile / tn) % tn, Tc = tile % tn;
      const int ua = Ta + j / 9 - 1, ub = Tb + (j / 3) % 3 - 1, uc = Tc + j % 3 - 1;
      nbase[u][j] = (ua >= 0 && ua < tn && ub >= 0 && ub < tn && uc >= 0 && uc < tn)
                        ? st.tile_base[(ua * tn + ub) * tn + uc] : -1;
    }
  }
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // half-wavefront h takes tiles h, h + 2, ...; its 32 lanes the pairs of
  // sub-grid rows (pi, 2 pjp) and (pi, 2 pjp + 1) at column pk
  const int h = lane >> 5, m = lane & 31;
  const int pi = m >> 3, pjp = (m >> 2) & 1, pk = m & 3;
  const int pos = 16 * pi + 8 * pjp + pk;   // the second row is pos + 4
  bool active[NL][2];
  int64_t row[NL][2];
  typename Epi::PreS pre[NL][2];
  bool any = false;
#pragma unroll
  for (int v = 0; v < NL; ++v) {
    const int u = h + 2 * v;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      active[v][r] = u < nt && ((st.mask[8 * (b0 + u) + t] >> (pos + 4 * r)) & 1);
      row[v][r] = u < nt ? static_cast<int64_t>(nbase[u][13]) + 64 * t + pos + 4 * r : 0;
      pre[v][r] = {};
      if (active[v][r]) pre[v][r] = epi.pre_s(row[v][r]);
      any = any || active[v][r];
    }
  }
  XT hv[NT][4];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (u >= nt) break;
    const int32_t tile = st.tiles[b0 + u];
    const int Ta = tile / (tn * tn), Tb = (tile / tn) % tn, Tc = tile % tn;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 512 * q;
      hv[u][q] = 0;
      if (e >= 1728) break;
      const int tp = e / 216, r = e - 216 * tp;
      const int I = r / 36, J = (r / 6) % 6, K = r % 6;
      const int a = 8 * Ta - 2 + (tp >> 2) + 2 * I;
      const int bb = 8 * Tb - 2 + ((tp >> 1) & 1) + 2 * J;
      const int c = 8 * Tc - 2 + (tp & 1) + 2 * K;
      if (a >= 0 && a < N && bb >= 0 && bb < N && c >= 0 && c < N) {
        const int32_t base = nbase[u][((a >> 3) - Ta + 1) * 9 + ((bb >> 3) - Tb + 1) * 3 + ((c >> 3) - Tc + 1)];
        if (base >= 0) hv[u][q] = x[base + 64 * tp + 16 * ((a & 7) >> 1) + 4 * ((bb & 7) >> 1) + ((c & 7) >> 1)];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (u >= nt) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 512 * q;
      if (e >= 1728) break;
      const int tp = e / 216, r = e - 216 * tp;
      halo[u * TILE + tp * STENCIL_SUB + (r / 36) * STENCIL_P1 + ((r / 6) % 6) * STENCIL_P2 + r % 6] = hv[u][q];
    }
  }
  __syncthreads();
  if (!any) return;
  const XT *hp = halo + h * TILE + pi * STENCIL_P1 + 2 * pjp * STENCIL_P2 + pk;
  const VT *val = st.val + 128 * t;
  using AT = typename Epi::acc_t;
  AT acc[NL][2];
  if (st.standard) {
    switch (t) {
      case 0: stencil_pairs_std<0, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      case 1: stencil_pairs_std<1, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      case 2: stencil_pairs_std<2, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      case 3: stencil_pairs_std<3, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      case 4: stencil_pairs_std<4, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      case 5: stencil_pairs_std<5, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      case 6: stencil_pairs_std<6, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
      default: stencil_pairs_std<7, NL, 2 * TILE, VT, XT, AT>(hp, val, acc); break;
    }
  } else {
    const int len = st.len[t];
    const int32_t *off = st.off + 128 * t;
#pragma unroll
    for (int v = 0; v < NL; ++v) acc[v][0] = acc[v][1] = 0;
    for (int j = 0; j < len; ++j) {
      const AT w = static_cast<AT>(val[j]);
#pragma unroll
      for (int v = 0; v < NL; ++v)
#pragma unroll
        for (int r = 0; r < 2; ++r) acc[v][r] += w * static_cast<AT>(hp[2 * v * TILE + off[j] + r * STENCIL_P2]);
    }
  }
  const AT dv = static_cast<AT>(st.dinv[t]);
#pragma unroll
  for (int v = 0; v < NL; ++v)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!active[v][r]) continue;
      const XT xi = hp[2 * v * TILE + r * STENCIL_P2 + t * STENCIL_SUB + STENCIL_P1 + STENCIL_P2 + 1];
      epi.apply_s(row[v][r], acc[v][r], pre[v][r], static_cast<AT>(xi), dv);
    }
}

template <typename VT, typename XT, class Epi>
static void launch_sell(const DevSELLView<VT> &A, const XT *x, Epi epi, hipStream_t s) {
  if (A.st.ntiles > 0) {
    if (A.st.ev0) (void)hipEventRecord(A.st.ev0, s);
    const unsigned wgs = static_cast<unsigned>((A.st.ntiles + STENCIL_TPW - 1) / STENCIL_TPW);
    stencil_kernel<VT, XT, Epi><<<wgs, 512, 0, s>>>(A.st, x, epi);
    if (A.st.ev1) (void)hipEventRecord(A.st.ev1, s);
  }
  if (A.nslices == 0) return;
  if (A.split) {
    const dim3 grid(static_cast<unsigned>((A.n * SELL_SPLIT + 255) / 256));
    sell_split_kernel<VT, XT, Epi><<<grid, 256, 0, s>>>(A.n, A.sl, A.cp, A.ci, A.bt, A.c16, A.btab, A.vp, A.v,
                                                        A.tid, A.tv, A.tw, A.rowmap, x, epi);
    return;
  }
  const dim3 grid(static_cast<unsigned>((A.nslices + SELL_WAVES - 1) / SELL_WAVES));
  sell_kernel<VT, XT, Epi><<<grid, 64 * SELL_WAVES, 0, s>>>(A.n, A.nslices, A.sl, A.cp, A.ci, A.bt, A.c16, A.btab,
                                                            A.vp, A.v, A.tid, A.tv, A.tw, A.rowmap, x, epi);
}

template <typename T>
void spmv(const DevSELLView<T> &A, const T *x, T *y, hipStream_t s) {
  launch_sell(A, x, EpiStore<T>{y}, s);
}
template <typename T>
void residual(const DevSELLView<T> &A, const T *x, const T *b, T *r, hipStream_t s) {
  launch_sell(A, x, EpiResidual<T>{b, r}, s);
}
template <typename T>
void cheb_step(const DevSELLView<T> &A, const T *b, const T *dinv, const T *xin, T *d, T *xout, T ca, T cb,
               hipStream_t s) {
  launch_sell(A, xin, EpiCheb<T>{b, dinv, xin, d, xout, ca, cb}, s);
}
template <typename T>
void spmv_add(const DevSELLView<T> &A, const T *x, T *y, hipStream_t s) {
  launch_sell(A, x, EpiAdd<T>{y}, s);
}
template void spmv_add<double>(const DevSELLView<double> &, const double *, double *, hipStream_t);
template void spmv_add<float>(const DevSELLView<float> &, const float *, float *, hipStream_t);
template void spmv<double>(const DevSELLView<double> &, const double *, double *, hipStream_t);
template void spmv<float>(const DevSELLView<float> &, const float *, float *, hipStream_t);
template void residual<double>(const DevSELLView<double> &, const double *, const double *, double *,
                               hipStream_t);
template void residual<float>(const DevSELLView<float> &, const float *, const float *, float *, hipStream_t);
template void cheb_step<double>(const DevSELLView<double> &, const double *, const double *, const double *,
                                double *, double *, double, double, hipStream_t);
template void cheb_step<float>(const DevSELLView<float> &, const float *, const float *, const float *, float *,
                               float *, float, float, hipStream_t);

}  // namespace fvem
