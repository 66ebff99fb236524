// Particle transfers and advection around the pressure solve (Algorithm 1,
// Sec. 3.2-3.3).  Every kernel is one thread per particle or per vertex and
// deterministic: sums run in a fixed order (P2G visits neighbour cells in a
// fixed order and each cell's particles by increasing index).
#include "transport.hpp"

#include <stdexcept>
#include <string>

namespace fvem {

namespace {

constexpr int TPB = 256;
constexpr int P2G_MAX_FIELDS = 8;
constexpr int LOCATE_MAX_DEPTH = 1 << 16;   // bound on a BSP descent (trees are finite)
constexpr int REFLECT_MAX = 4;

inline void launch_check(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

inline unsigned grid_of(int64_t n) { return static_cast<unsigned>((n + TPB - 1) / TPB); }

__device__ inline int64_t bg_index(const TransportView &T, double x, double y, double z) {
  const int N = T.N;
  const int i = min(max(static_cast<int>(floor(x * N)), 0), N - 1);
  const int j = min(max(static_cast<int>(floor(y * N)), 0), N - 1);
  const int k = min(max(static_cast<int>(floor(z * N)), 0), N - 1);
  return (static_cast<int64_t>(i) * N + j) * N + k;
}

// level-0 cell holding the point: the background cell's cube cell, or the
// leaf of its BSP tree reached by the split planes
__device__ int32_t locate_point(const TransportView &T, double x, double y, double z) {
  if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0 && z >= 0.0 && z <= 1.0)) return -1;
  const int32_t v = T.bg[bg_index(T, x, y, z)];
  if (v >= -1) return v;
  int32_t nd = T.tree_root[-2 - v];
  for (int depth = 0; depth < LOCATE_MAX_DEPTH && T.child[2 * nd] >= 0; ++depth) {
    const double *p = T.plane + 4 * static_cast<int64_t>(nd);
    nd = (p[0] * x + p[1] * y + p[2] * z < p[3]) ? T.child[2 * nd] : T.child[2 * nd + 1];
  }
  return T.child[2 * nd] >= 0 ? -1 : T.leaf_cell[nd];
}

// cell c's linear velocity at (x, y, z): 3 components on [1, (x - x_E)/h_E]
__device__ inline void eval_cell(const TransportView &T, const double *sf, int32_t c, const double *x, double *u) {
  const double *g = T.cell_geom + 5 * static_cast<int64_t>(c);
  const double inv = 1.0 / g[3];
  const double z0 = (x[0] - g[0]) * inv, z1 = (x[1] - g[1]) * inv, z2 = (x[2] - g[2]) * inv;
  const double *s = sf + 12 * static_cast<int64_t>(c);
  for (int d = 0; d < 3; ++d) u[d] = s[4 * d] + s[4 * d + 1] * z0 + s[4 * d + 2] * z1 + s[4 * d + 3] * z2;
}

__global__ void locate_kernel(TransportView T, int64_t n, const double *x, int32_t *cell) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) cell[p] = locate_point(T, x[3 * p], x[3 * p + 1], x[3 * p + 2]);
}

// ------------------------------------------------------------------ P2G

__global__ void count_kernel(TransportView T, int64_t n, const double *x, int32_t *count) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) atomicAdd(&count[bg_index(T, x[3 * p], x[3 * p + 1], x[3 * p + 2])], 1);
}

__global__ void fill_kernel(int32_t *a, int64_t m) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) a[i] = 0;
}

// exclusive scan of count[0 .. m) into start[0 .. m] in three passes: chunk
// sums, a scan of the chunk sums (one block), and the chunks rescanned from
// their offsets
constexpr int SCAN_THREADS = 1024, SCAN_ITEMS = 8, SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

__device__ int32_t block_exclusive_scan(int32_t v, int32_t *buf, int32_t *total) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    const int32_t t = threadIdx.x >= static_cast<unsigned>(off) ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += t;
    __syncthreads();
  }
  const int32_t incl = buf[threadIdx.x];
  *total = buf[SCAN_THREADS - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void chunk_sum_kernel(const int32_t *count, int64_t m, int32_t *chunk) {
  __shared__ int32_t buf[SCAN_THREADS];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_CHUNK + static_cast<int64_t>(threadIdx.x) * SCAN_ITEMS;
  int32_t v = 0;
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < m) v += count[base + q];
  int32_t total;
  block_exclusive_scan(v, buf, &total);
  if (threadIdx.x == 0) chunk[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void chunk_scan_kernel(int32_t *chunk, int64_t nchunk) {
  __shared__ int32_t buf[SCAN_THREADS];
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nchunk; b0 += SCAN_THREADS) {
    const int64_t i = b0 + threadIdx.x;
    const int32_t v = i < nchunk ? chunk[i] : 0;
    int32_t total;
    const int32_t ex = block_exclusive_scan(v, buf, &total);
    if (i < nchunk) chunk[i] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(SCAN_THREADS) void chunk_apply_kernel(const int32_t *count, int64_t m,
                                                                   const int32_t *chunk, int32_t *start) {
  __shared__ int32_t buf[SCAN_THREADS];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_CHUNK + static_cast<int64_t>(threadIdx.x) * SCAN_ITEMS;
  int32_t v = 0;
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < m) v += count[base + q];
  int32_t total;
  int32_t run = chunk[blockIdx.x] + block_exclusive_scan(v, buf, &total);
  for (int q = 0; q < SCAN_ITEMS; ++q)
    if (base + q < m) {
      start[base + q] = run;
      run += count[base + q];
    }
  if (base + SCAN_ITEMS >= m && base < m) start[m] = run;   // the thread holding the last element
}

__global__ void scatter_kernel(TransportView T, int64_t n, const double *x, const int32_t *start, int32_t *cursor,
                               int32_t *order) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t b = bg_index(T, x[3 * p], x[3 * p + 1], x[3 * p + 2]);
  order[start[b] + atomicAdd(&cursor[b], 1)] = static_cast<int32_t>(p);
}

// each background cell's particles by increasing index (the scatter order
// depends on atomic timing)
__global__ void sort_cells_kernel(int64_t m, const int32_t *start, int32_t *order) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= m) return;
  const int32_t s0 = start[b], s1 = start[b + 1];
  for (int32_t i = s0 + 1; i < s1; ++i) {
    const int32_t v = order[i];
    int32_t j = i - 1;
    while (j >= s0 && order[j] > v) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
}

__global__ void gather_kernel(TransportView T, const double *x, const double *f, int m, const int32_t *start,
                              const int32_t *order, double *out) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= T.n_vert) return;
  const double xi = T.vert_xyz[3 * v], yi = T.vert_xyz[3 * v + 1], zi = T.vert_xyz[3 * v + 2];
  const int N = T.N;
  const int ci = min(max(static_cast<int>(floor(xi * N)), 0), N - 1);
  const int cj = min(max(static_cast<int>(floor(yi * N)), 0), N - 1);
  const int ck = min(max(static_cast<int>(floor(zi * N)), 0), N - 1);
  const double inv_r2 = static_cast<double>(N) * N;   // R = h
  double acc[P2G_MAX_FIELDS];
  for (int a = 0; a < P2G_MAX_FIELDS; ++a) acc[a] = 0.0;
  double sw = 0.0;
  for (int i = max(ci - 1, 0); i <= min(ci + 1, N - 1); ++i)
    for (int j = max(cj - 1, 0); j <= min(cj + 1, N - 1); ++j)
      for (int k = max(ck - 1, 0); k <= min(ck + 1, N - 1); ++k) {
        const int64_t b = (static_cast<int64_t>(i) * N + j) * N + k;
        for (int32_t q = start[b]; q < start[b + 1]; ++q) {
          const int64_t p = order[q];
          const double dx = x[3 * p] - xi, dy = x[3 * p + 1] - yi, dz = x[3 * p + 2] - zi;
          const double qq = (dx * dx + dy * dy + dz * dz) * inv_r2;
          if (qq >= 1.0) continue;
          const double om = 1.0 - qq, w = om * om * om;
          sw += w;
          for (int a = 0; a < m; ++a) acc[a] += w * f[p * m + a];
        }
      }
  for (int a = 0; a < m; ++a) out[v * m + a] = sw > 0.0 ? acc[a] / sw : 0.0;
}

__global__ void buoyancy_kernel(int64_t nv, const double *f, int m, double alpha, double beta, double dt, double *u) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const double *r = f + v * m;
  u[3 * v] = r[0];
  u[3 * v + 1] = r[1];
  u[3 * v + 2] = r[2] + dt * (-alpha * r[3] + beta * r[4]);
}

// ------------------------------------------------------------------ G2P

__global__ void g2p_kernel(TransportView T, int64_t n, const double *x, const uint8_t *ghost, double *u,
                           const double *s_new, const double *s_old, double a) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n || ghost[p]) return;
  const double xp[3] = {x[3 * p], x[3 * p + 1], x[3 * p + 2]};
  const int32_t c = locate_point(T, xp[0], xp[1], xp[2]);
  if (c < 0) return;
  double un[3], uo[3];
  eval_cell(T, s_new, c, xp, un);
  eval_cell(T, s_old, c, xp, uo);
  for (int d = 0; d < 3; ++d) u[3 * p + d] = a * (u[3 * p + d] + (un[d] - uo[d])) + (1.0 - a) * un[d];
}

__global__ void speed_kernel(TransportView T, int64_t n, const double *x, const uint8_t *ghost, const double *sf,
                             unsigned long long *vmax) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n || ghost[p]) return;
  const double xp[3] = {x[3 * p], x[3 * p + 1], x[3 * p + 2]};
  const int32_t c = locate_point(T, xp[0], xp[1], xp[2]);
  if (c < 0) return;
  double u[3];
  eval_cell(T, sf, c, xp, u);
  const double v = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  // non-negative doubles order like their bit patterns
  atomicMax(vmax, static_cast<unsigned long long>(__double_as_longlong(v)));
}

// ------------------------------------------------------------ advection

struct Hit {
  double t = 2.0;
  double n[3] = {0.0, 0.0, 0.0};
  int32_t tri = -1;
};

// first point where the segment a -> a + d leaves the unit box or meets a
// boundary triangle listed in a background cell its bounding box touches
__device__ Hit first_crossing(const TransportView &T, const double *a, const double *d) {
  Hit h;
  for (int ax = 0; ax < 3; ++ax)
    for (int w = 0; w < 2; ++w)
      if (d[ax] != 0.0) {
        const double t = (static_cast<double>(w) - a[ax]) / d[ax];
        if (t > 1e-12 && t <= 1.0 && t < h.t) {
          h.t = t;
          h.n[0] = h.n[1] = h.n[2] = 0.0;
          h.n[ax] = 1.0;
          h.tri = -1;
        }
      }
  const int N = T.N;
  int lo[3], hi[3];
  for (int ax = 0; ax < 3; ++ax) {
    const double e0 = a[ax], e1 = a[ax] + d[ax];
    lo[ax] = min(max(static_cast<int>(floor(fmin(e0, e1) * N)), 0), N - 1);
    hi[ax] = min(max(static_cast<int>(floor(fmax(e0, e1) * N)), 0), N - 1);
  }
  for (int i = lo[0]; i <= hi[0]; ++i)
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int k = lo[2]; k <= hi[2]; ++k) {
        const int64_t b = (static_cast<int64_t>(i) * N + j) * N + k;
        for (int64_t q = T.tri_ptr[b]; q < T.tri_ptr[b + 1]; ++q) {
          const int32_t tid = T.tri_id[q];
          const double *P = T.tri_xyz + 9 * static_cast<int64_t>(tid);
          const double e1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
          const double e2[3] = {P[6] - P[0], P[7] - P[1], P[8] - P[2]};
          const double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
          const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
          if (!(fabs(det) > 1e-300)) continue;
          const double inv = 1.0 / det;
          const double tv[3] = {a[0] - P[0], a[1] - P[1], a[2] - P[2]};
          const double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
          const double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
          const double v = (qv[0] * d[0] + qv[1] * d[1] + qv[2] * d[2]) * inv;
          const double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
          if (!(u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t > 1e-12 && t <= 1.0)) continue;
          // the earliest crossing; a wall wins a tie, then the lower triangle
          if (!(t < h.t || (t == h.t && h.tri >= 0 && tid < h.tri))) continue;
          const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                       cz = e1[0] * e2[1] - e1[1] * e2[0];
          const double nn = sqrt(cx * cx + cy * cy + cz * cz);
          h.t = t;
          h.n[0] = cx / nn;
          h.n[1] = cy / nn;
          h.n[2] = cz / nn;
          h.tri = tid;
        }
      }
  return h;
}

// end of a stage a -> b: b if it is in the fluid, else b mirrored in the
// plane of the first boundary crossing (at most REFLECT_MAX times); a point
// still outside falls back to the stage's start
__device__ void resolve(const TransportView &T, const double *a_in, double *b) {
  double a[3] = {a_in[0], a_in[1], a_in[2]};
  for (int it = 0; it < REFLECT_MAX; ++it) {
    if (locate_point(T, b[0], b[1], b[2]) >= 0) return;
    const double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const Hit h = first_crossing(T, a, d);
    if (h.t > 1.0) {
      b[0] = a_in[0], b[1] = a_in[1], b[2] = a_in[2];
      return;
    }
    const double q[3] = {a[0] + h.t * d[0], a[1] + h.t * d[1], a[2] + h.t * d[2]};
    const double s = (b[0] - q[0]) * h.n[0] + (b[1] - q[1]) * h.n[1] + (b[2] - q[2]) * h.n[2];
    for (int ax = 0; ax < 3; ++ax) {
      b[ax] -= 2.0 * s * h.n[ax];
      a[ax] = q[ax];
    }
  }
  if (locate_point(T, b[0], b[1], b[2]) < 0) b[0] = a_in[0], b[1] = a_in[1], b[2] = a_in[2];
}

__device__ inline void velocity_at(const TransportView &T, const double *sf, const double *y, double *u) {
  const int32_t c = locate_point(T, y[0], y[1], y[2]);
  if (c < 0) {
    u[0] = u[1] = u[2] = 0.0;
    return;
  }
  eval_cell(T, sf, c, y, u);
}

__global__ void advect_kernel(TransportView T, int64_t n, double *x, const uint8_t *ghost, const double *sf,
                              double tau, int n_sub) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n || ghost[p]) return;
  double a[3] = {x[3 * p], x[3 * p + 1], x[3 * p + 2]};
  for (int s = 0; s < n_sub; ++s) {
    if (locate_point(T, a[0], a[1], a[2]) < 0) continue;
    double u[3], mid[3], end[3];
    velocity_at(T, sf, a, u);
    for (int d = 0; d < 3; ++d) mid[d] = a[d] + 0.5 * tau * u[d];
    resolve(T, a, mid);
    velocity_at(T, sf, mid, u);
    for (int d = 0; d < 3; ++d) end[d] = a[d] + tau * u[d];
    resolve(T, a, end);
    for (int d = 0; d < 3; ++d) a[d] = end[d];
  }
  for (int d = 0; d < 3; ++d) x[3 * p + d] = a[d];
}

}  // namespace

void locate(const TransportView &T, int64_t n, const double *x, int32_t *cell, hipStream_t s) {
  if (n <= 0) return;
  locate_kernel<<<grid_of(n), TPB, 0, s>>>(T, n, x, cell);
  launch_check("locate");
}

int64_t p2g_chunks(int32_t N) {
  const int64_t N3 = static_cast<int64_t>(N) * N * N;
  return (N3 + SCAN_CHUNK - 1) / SCAN_CHUNK;
}

void p2g(const TransportView &T, int64_t n, const double *x, const double *f, int m, double *out,
         int32_t *cell_count, int32_t *cell_start, int32_t *chunk, int32_t *order, hipStream_t s) {
  if (m < 1 || m > P2G_MAX_FIELDS) throw std::runtime_error("p2g: 1 to 8 fields per particle");
  const int64_t N3 = static_cast<int64_t>(T.N) * T.N * T.N;
  const int64_t nchunk = p2g_chunks(T.N);
  fill_kernel<<<grid_of(N3 + 1), TPB, 0, s>>>(cell_count, N3 + 1);
  if (n > 0) count_kernel<<<grid_of(n), TPB, 0, s>>>(T, n, x, cell_count);
  chunk_sum_kernel<<<static_cast<unsigned>(nchunk), SCAN_THREADS, 0, s>>>(cell_count, N3, chunk);
  chunk_scan_kernel<<<1, SCAN_THREADS, 0, s>>>(chunk, nchunk);
  chunk_apply_kernel<<<static_cast<unsigned>(nchunk), SCAN_THREADS, 0, s>>>(cell_count, N3, chunk, cell_start);
  fill_kernel<<<grid_of(N3 + 1), TPB, 0, s>>>(cell_count, N3 + 1);
  if (n > 0) scatter_kernel<<<grid_of(n), TPB, 0, s>>>(T, n, x, cell_start, cell_count, order);
  sort_cells_kernel<<<grid_of(N3), TPB, 0, s>>>(N3, cell_start, order);
  if (T.n_vert > 0) gather_kernel<<<grid_of(T.n_vert), TPB, 0, s>>>(T, x, f, m, cell_start, order, out);
  launch_check("p2g");
}

void buoyancy(int64_t n_vert, const double *f, int m, double alpha, double beta, double dt, double *u_out,
              hipStream_t s) {
  if (m < 5) throw std::runtime_error("buoyancy: fields are u (3), density, temperature");
  if (n_vert <= 0) return;
  buoyancy_kernel<<<grid_of(n_vert), TPB, 0, s>>>(n_vert, f, m, alpha, beta, dt, u_out);
  launch_check("buoyancy");
}

void g2p(const TransportView &T, int64_t n, const double *x, const uint8_t *ghost, double *u, const double *s_new,
         const double *s_old, double a_flip, hipStream_t s) {
  if (n <= 0) return;
  g2p_kernel<<<grid_of(n), TPB, 0, s>>>(T, n, x, ghost, u, s_new, s_old, a_flip);
  launch_check("g2p");
}

void grid_speed_max(const TransportView &T, int64_t n, const double *x, const uint8_t *ghost, const double *sf,
                    unsigned long long *vmax_bits, hipStream_t s) {
  if (n <= 0) return;
  speed_kernel<<<grid_of(n), TPB, 0, s>>>(T, n, x, ghost, sf, vmax_bits);
  launch_check("grid speed");
}

void advect(const TransportView &T, int64_t n, double *x, const uint8_t *ghost, const double *sf, double dt,
            int n_sub, hipStream_t s) {
  if (n <= 0 || n_sub < 1) return;
  advect_kernel<<<grid_of(n), TPB, 0, s>>>(T, n, x, ghost, sf, dt / n_sub, n_sub);
  launch_check("advect");
}

}  // namespace fvem
