// Level-0 operators applied cell by cell from their element blocks.  One
// thread per cell forms the cell's local products; outputs owned by one cell
// (cell fields) are written directly, outputs shared by several cells
// (pressure DOFs, vertex velocities) go to per-cell slots of a scratch array
// and are then summed per output over its slots in increasing order.  No
// atomics, so every result is bitwise reproducible.
#include "elem.hpp"

#include <stdexcept>
#include <string>

namespace fvem {

namespace {

constexpr int TPB = 256;

inline unsigned grid_of(int64_t n) { return static_cast<unsigned>((n + TPB - 1) / TPB); }

__device__ inline void put(double *y, int64_t i, double v, bool acc, double scale) {
  y[i] = acc ? y[i] + scale * v : scale * v;
}

__device__ inline double za(const ElemView &E, const double *g, int32_t vtx, int a) {
  return a == 0 ? 1.0 : (E.xyz[3 * static_cast<int64_t>(vtx) + a - 1] - g[a - 1]) / g[3];
}

template <ElemOp OP>
__global__ void cell_kernel(ElemView E, const double *x, double *y, bool acc, double scale) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= E.ncell) return;
  const int64_t p0 = E.cptr[c], nE = E.cptr[c + 1] - p0;
  const int64_t v0 = E.vptr[c], nvE = E.vptr[c + 1] - v0;
  const int32_t *cd = E.cdof + p0;
  const int32_t *cv = E.vert + v0;
  if constexpr (OP == ELEM_B || OP == ELEM_BT) {
    const double *be = E.be_val + E.be_off[c];
    const int64_t w = 3 * nvE;
    if constexpr (OP == ELEM_B) {
      for (int64_t q = 0; q < nE; ++q) {
        double a = 0.0;
        for (int64_t v = 0; v < nvE; ++v) {
          const double *u = x + 3 * static_cast<int64_t>(cv[v]);
          const double *r = be + q * w + 3 * v;
          a += r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
        }
        E.tmp[p0 + q] = a;
      }
    } else {
      for (int64_t v = 0; v < nvE; ++v)
        for (int d = 0; d < 3; ++d) {
          double a = 0.0;
          for (int64_t q = 0; q < nE; ++q)
            if (cd[q] >= 0) a += be[q * w + 3 * v + d] * x[cd[q]];
          E.tmp[3 * (v0 + v) + d] = a;
        }
    }
    return;
  } else {
    const double *blk = E.vc_val + E.vc_off[c];
    const double *pi1 = blk, *gk = blk + 4 * nvE, *m1 = blk + 4 * nvE + 12 * nE;
    const double *g = E.geom + 5 * c;
    if constexpr (OP == ELEM_PI) {
      for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 4; ++a) {
          double s = 0.0;
          for (int64_t v = 0; v < nvE; ++v) s += pi1[a * nvE + v] * x[3 * static_cast<int64_t>(cv[v]) + d];
          put(y, 12 * c + 4 * d + a, s, acc, scale);
        }
    } else if constexpr (OP == ELEM_PIT) {
      for (int64_t v = 0; v < nvE; ++v)
        for (int d = 0; d < 3; ++d) {
          double s = 0.0;
          for (int a = 0; a < 4; ++a) s += pi1[a * nvE + v] * x[12 * c + 4 * d + a];
          E.tmp[3 * (v0 + v) + d] = s;
        }
    } else if constexpr (OP == ELEM_G) {
      for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 4; ++a) {
          double s = 0.0;
          for (int64_t q = 0; q < nE; ++q)
            if (cd[q] >= 0) s += gk[(4 * d + a) * nE + q] * x[cd[q]];
          put(y, 12 * c + 4 * d + a, s, acc, scale);
        }
    } else if constexpr (OP == ELEM_GT) {
      for (int64_t q = 0; q < nE; ++q) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d)
          for (int a = 0; a < 4; ++a) s += gk[(4 * d + a) * nE + q] * x[12 * c + 4 * d + a];
        E.tmp[p0 + q] = s;
      }
    } else if constexpr (OP == ELEM_M) {
      for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 4; ++a) {
          double s = 0.0;
          for (int b = 0; b < 4; ++b) s += m1[a * 4 + b] * x[12 * c + 4 * d + b];
          put(y, 12 * c + 4 * d + a, s, acc, scale);
        }
    } else if constexpr (OP == ELEM_AVT) {
      for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 4; ++a) {
          double s = 0.0;
          for (int64_t v = 0; v < nvE; ++v)
            s += g[4] * E.winv[cv[v]] * za(E, g, cv[v], a) * x[3 * static_cast<int64_t>(cv[v]) + d];
          put(y, 12 * c + 4 * d + a, s, acc, scale);
        }
    } else {   // ELEM_AV: the cell's volume-weighted polynomial at its vertices
      for (int64_t v = 0; v < nvE; ++v)
        for (int d = 0; d < 3; ++d) {
          double s = 0.0;
          for (int a = 0; a < 4; ++a) s += za(E, g, cv[v], a) * x[12 * c + 4 * d + a];
          E.tmp[3 * (v0 + v) + d] = g[4] * s;
        }
    }
  }
}

// pressure slot i: the sum of its cells' contributions
__global__ void sum_pressure_kernel(ElemView E, double *y, bool acc, double scale) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= E.nl) return;
  double a = 0.0;
  for (int64_t k = E.pptr[i]; k < E.pptr[i + 1]; ++k) a += E.tmp[E.ppos[k]];
  put(y, i, a, acc, scale);
}

// vertex component 3 v + d: the sum of its cells' contributions, scaled by
// 1 / (volume around v) for the vertex average
__global__ void sum_vertex_kernel(ElemView E, double *y, bool acc, double scale, bool average) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 3 * E.nv) return;
  const int64_t v = i / 3;
  const int d = static_cast<int>(i - 3 * v);
  double a = 0.0;
  for (int64_t k = E.qptr[v]; k < E.qptr[v + 1]; ++k) a += E.tmp[3 * static_cast<int64_t>(E.qpos[k]) + d];
  if (average) a *= E.winv[v];
  put(y, i, a, acc, scale);
}

template <ElemOp OP>
void launch_cells(const ElemView &E, const double *x, double *y, bool acc, double scale, hipStream_t s) {
  cell_kernel<OP><<<grid_of(E.ncell), TPB, 0, s>>>(E, x, y, acc, scale);
}

}  // namespace

void elem_apply(const ElemView &E, ElemOp op, const double *x, double *y, bool accumulate, double scale,
                hipStream_t s) {
  const bool velocity_op = op != ELEM_B && op != ELEM_BT;
  if (velocity_op && !E.vc_off) throw std::runtime_error("no velocity blocks");
  if (!velocity_op && !E.be_off) throw std::runtime_error("no divergence blocks");
  if (E.ncell > 0) {
    switch (op) {
      case ELEM_B: launch_cells<ELEM_B>(E, x, y, accumulate, scale, s); break;
      case ELEM_BT: launch_cells<ELEM_BT>(E, x, y, accumulate, scale, s); break;
      case ELEM_PI: launch_cells<ELEM_PI>(E, x, y, accumulate, scale, s); break;
      case ELEM_PIT: launch_cells<ELEM_PIT>(E, x, y, accumulate, scale, s); break;
      case ELEM_G: launch_cells<ELEM_G>(E, x, y, accumulate, scale, s); break;
      case ELEM_GT: launch_cells<ELEM_GT>(E, x, y, accumulate, scale, s); break;
      case ELEM_M: launch_cells<ELEM_M>(E, x, y, accumulate, scale, s); break;
      case ELEM_AV: launch_cells<ELEM_AV>(E, x, y, accumulate, scale, s); break;
      case ELEM_AVT: launch_cells<ELEM_AVT>(E, x, y, accumulate, scale, s); break;
    }
  }
  if (op == ELEM_B || op == ELEM_GT) {
    if (E.nl > 0) sum_pressure_kernel<<<grid_of(E.nl), TPB, 0, s>>>(E, y, accumulate, scale);
  } else if (op == ELEM_BT || op == ELEM_PIT || op == ELEM_AV) {
    if (E.nv > 0) sum_vertex_kernel<<<grid_of(3 * E.nv), TPB, 0, s>>>(E, y, accumulate, scale, op == ELEM_AV);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("element operator: ") + hipGetErrorString(e));
}

}  // namespace fvem
