// Level-0 operators applied cell by cell from their element blocks
// (implemented in elem.hip): the divergence B (Sec. 3.2 right-hand side) and
// the velocity operators of the Sec. 3.3 correction.  Cells of one shape
// share a block, so the operators cost a block offset and index lists per
// cell instead of stored nonzeros (the compact storage of regular regions).
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace fvem {

// Cell-field vectors hold 12 values per cell: velocity component d, monomial
// a of [1, (x - x_E)/h_E] at 12 c + 4 d + a.  Pressure vectors are in the
// level order (nl entries, holes included); velocity vectors hold 3 values
// per vertex.
struct ElemView {
  int64_t ncell = 0, nl = 0, nv = 0;
  const int64_t *cptr = nullptr;   // ncell + 1: pressure DOFs of each cell
  const int32_t *cdof = nullptr;   // their level-order slots, -1 eliminated
  const int64_t *vptr = nullptr;   // ncell + 1: velocity vertices of each cell
  const int32_t *vert = nullptr;
  const int64_t *be_off = nullptr; // divergence block, n_E x 3 n_vE row-major (column 3 v + d)
  const double *be_val = nullptr;
  const int64_t *vc_off = nullptr; // Pi_1 (4 x n_vE), grad Pi_k (3 x 4 x n_E), M1 (4 x 4); NULL without
  const double *vc_val = nullptr;
  const double *geom = nullptr;    // 5 per cell: centroid, h_E, volume
  const double *xyz = nullptr;     // 3 per vertex
  const double *winv = nullptr;    // per vertex: 1 / (volume of the cells around it)
  // positions of each pressure slot in cdof and of each vertex in vert, in
  // increasing order (the fixed summation order of shared outputs)
  const int64_t *pptr = nullptr;   // nl + 1
  const int32_t *ppos = nullptr;
  const int64_t *qptr = nullptr;   // nv + 1
  const int32_t *qpos = nullptr;
  double *tmp = nullptr;           // max(cptr[ncell], 3 vptr[ncell]) doubles
};

enum ElemOp {
  ELEM_B,     // b = B u             (pressure <- velocity)
  ELEM_BT,    // u = B^T b           (velocity <- pressure)
  ELEM_PI,    // s = Pi_1 u          (cell field <- velocity)
  ELEM_PIT,   // u = Pi_1^T s
  ELEM_G,     // s = grad Pi_k p     (cell field <- pressure)
  ELEM_GT,    // p = (grad Pi_k)^T s
  ELEM_M,     // s = blockdiag(M1) t (cell field <- cell field)
  ELEM_AV,    // u = Av s: volume-weighted vertex average of the cell polynomials
  ELEM_AVT    // s = Av^T u
};

// y = scale * op(x), or y += scale * op(x) with accumulate
void elem_apply(const ElemView &E, ElemOp op, const double *x, double *y, bool accumulate, double scale,
                hipStream_t s);

}  // namespace fvem
