// Particle transfers and advection around the pressure solve (Algorithm 1,
// Sec. 3.2-3.3), implemented in transport.hip.
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace fvem {

// Finest-level geometry for point location and collision (device pointers).
struct TransportView {
  int32_t N = 0;                        // background grid N^3 on the unit cube
  const int32_t *bg = nullptr;          // N^3: level-0 cube cell, -1, or -2 - tree
  const int32_t *tree_root = nullptr;   // first node of each BSP tree
  const double *plane = nullptr;        // 4 per node: n, d (inner nodes)
  const int32_t *child = nullptr;       // 2 per node: n.x < d, n.x >= d; -1 at leaves
  const int32_t *leaf_cell = nullptr;   // per node: the leaf's level-0 cell or -1
  const int64_t *tri_ptr = nullptr;     // N^3 + 1: triangles per background cell
  const int32_t *tri_id = nullptr;
  const double *tri_xyz = nullptr;      // 9 per triangle
  const double *cell_geom = nullptr;    // 5 per level-0 cell: centroid, h_E, volume
  const double *vert_xyz = nullptr;     // 3 per velocity vertex
  int64_t n_vert = 0;
};

// level-0 cell of each point (-1: solid or outside the unit cube)
void locate(const TransportView &T, int64_t n, const double *x, int32_t *cell, hipStream_t s);

// P2G: out[i, :] = sum_p f[p, :] w_ip / sum_p w_ip over particles within h
// of vertex i (0 where none); cell_count, cell_start, chunk and order are
// scratch of N^3 + 1, N^3 + 1, p2g_chunks(N) and n entries
int64_t p2g_chunks(int32_t N);
void p2g(const TransportView &T, int64_t n, const double *x, const double *f, int m, double *out,
         int32_t *cell_count, int32_t *cell_start, int32_t *chunk, int32_t *order, hipStream_t s);

// u'[3 v + 2] = u[v, 2] + dt (-alpha f[v, 3] + beta f[v, 4]), u'[3 v + d] = f[v, d] otherwise
void buoyancy(int64_t n_vert, const double *f, int m, double alpha, double beta, double dt, double *u_out,
              hipStream_t s);

// FLIP/PIC update of non-ghost particle velocities from the cell fields
// s_new, s_old (12 per cell: 3 components x [1, (x - x_E)/h_E])
void g2p(const TransportView &T, int64_t n, const double *x, const uint8_t *ghost, double *u, const double *s_new,
         const double *s_old, double a_flip, hipStream_t s);

// largest grid speed |s(x_p)| over non-ghost particles, as the bits of a
// non-negative double in *vmax_bits (zeroed by the caller)
void grid_speed_max(const TransportView &T, int64_t n, const double *x, const uint8_t *ghost, const double *sf,
                    unsigned long long *vmax_bits, hipStream_t s);

// n_sub midpoint RK2 substeps of length dt / n_sub through the cell field sf,
// with mirror reflection at obstacle triangles and the box walls
void advect(const TransportView &T, int64_t n, double *x, const uint8_t *ghost, const double *sf, double dt,
            int n_sub, hipStream_t s);

}  // namespace fvem
