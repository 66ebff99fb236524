// Row epilogues of the SpMV kernels: what a kernel does with (A x)_i once a
// row's sum is complete (store, residual, prolong-and-correct, scaled store,
// fused Chebyshev step).  Shared by the CSR (kernels.hip) and sliced
// (sell.hip) SpMV kernels.
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace fvem {

// Each epilogue can also be split in two for kernels that overlap the
// row's own vector reads with their gathers: pre(i) issues the reads,
// apply(i, a, pre, x_i) finishes the row given x_i (x at the row itself).
// Lattice stencil rows share their class's diagonal, so the Chebyshev step
// takes D^-1 from the class there: pre_s / apply_s(..., dinv) skip its
// stream (the other epilogues do not read D^-1 and alias them).

template <typename T>
struct EpiStore {
  using acc_t = T;
  T *y;
  __device__ void operator()(int64_t i, T a) const { y[i] = a; }
  struct Pre {};
  __device__ Pre pre(int64_t) const { return {}; }
  __device__ void apply(int64_t i, T a, const Pre &, T) const { y[i] = a; }
  using PreS = Pre;
  __device__ PreS pre_s(int64_t i) const { return pre(i); }
  __device__ void apply_s(int64_t i, T a, const PreS &p, T x, T) const { apply(i, a, p, x); }
};

template <typename T>
struct EpiResidual {  // y = b - A x
  using acc_t = T;
  const T *b;
  T *y;
  __device__ void operator()(int64_t i, T a) const { y[i] = b[i] - a; }
  struct Pre { T b; };
  __device__ Pre pre(int64_t i) const { return {b[i]}; }
  __device__ void apply(int64_t i, T a, const Pre &p, T) const { y[i] = p.b - a; }
  using PreS = Pre;
  __device__ PreS pre_s(int64_t i) const { return pre(i); }
  __device__ void apply_s(int64_t i, T a, const PreS &p, T x, T) const { apply(i, a, p, x); }
};

template <typename T>
struct EpiAdd {  // y += A x  (prolong-and-correct)
  using acc_t = T;
  T *y;
  __device__ void operator()(int64_t i, T a) const { y[i] += a; }
  struct Pre { T y; };
  __device__ Pre pre(int64_t i) const { return {y[i]}; }
  __device__ void apply(int64_t i, T a, const Pre &p, T) const { y[i] = p.y + a; }
  using PreS = Pre;
  __device__ PreS pre_s(int64_t i) const { return pre(i); }
  __device__ void apply_s(int64_t i, T a, const PreS &p, T x, T) const { apply(i, a, p, x); }
};

struct EpiScaled {  // y = alpha A x
  using acc_t = double;
  double *y;
  double alpha;
  __device__ void operator()(int64_t i, double a) const { y[i] = alpha * a; }
};

template <typename T>
struct EpiCheb {  // d = ca d + cb dinv (b - A xin);  xout = xin + d
  using acc_t = T;
  const T *b, *dinv, *xin;
  T *d, *xout;
  T ca, cb;
  __device__ void operator()(int64_t i, T a) const {
    const T dn = ca * d[i] + cb * dinv[i] * (b[i] - a);
    d[i] = dn;
    xout[i] = xin[i] + dn;
  }
  struct Pre { T b, dinv, d; };
  __device__ Pre pre(int64_t i) const { return {b[i], dinv[i], d[i]}; }
  __device__ void apply(int64_t i, T a, const Pre &p, T x) const {
    const T dn = ca * p.d + cb * p.dinv * (p.b - a);
    d[i] = dn;
    xout[i] = x + dn;
  }
  struct PreS { T b, d; };
  __device__ PreS pre_s(int64_t i) const { return {b[i], d[i]}; }
  __device__ void apply_s(int64_t i, T a, const PreS &p, T x, T dv) const {
    const T dn = ca * p.d + cb * dv * (p.b - a);
    d[i] = dn;
    xout[i] = x + dn;
  }
};

}  // namespace fvem
