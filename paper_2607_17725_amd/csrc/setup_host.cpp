// Host-side hierarchy setup (see setup_host.hpp).
#include "setup_host.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <omp.h>

namespace fvem {

namespace {

// DOF -> (cell, local index) incidence, cells in increasing order per DOF.
void incidence(int64_t n, const HostCells &cells, std::vector<int64_t> &ptr, std::vector<int64_t> &cell,
               std::vector<int32_t> &loc) {
  ptr.assign(n + 1, 0);
  for (int64_t c = 0; c < cells.n_cells; ++c)
    for (int64_t k = cells.ptr[c]; k < cells.ptr[c + 1]; ++k)
      if (cells.dof[k] >= 0) ptr[cells.dof[k] + 1]++;
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  cell.resize(ptr[n]);
  loc.resize(ptr[n]);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t c = 0; c < cells.n_cells; ++c)
    for (int64_t k = cells.ptr[c]; k < cells.ptr[c + 1]; ++k) {
      int32_t d = cells.dof[k];
      if (d < 0) continue;
      cell[fill[d]] = c;
      loc[fill[d]] = static_cast<int32_t>(k - cells.ptr[c]);
      fill[d]++;
    }
}

}  // namespace

HostCSR assemble_blocks(int64_t n_rows, int64_t n_cols, const HostCells &rows, const HostCells &cols,
                        const HostBlocks &blocks) {
  std::vector<int64_t> iptr, icell;
  std::vector<int32_t> iloc;
  incidence(n_rows, rows, iptr, icell, iloc);
  HostCSR A;
  A.n_rows = n_rows;
  A.n_cols = n_cols;
  A.rp.assign(n_rows + 1, 0);
  // symbolic: sorted union of the column lists of the incident cells
  std::vector<std::vector<int32_t>> pat(n_rows);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n_rows; ++i) {
    std::vector<int32_t> &p = pat[i];
    for (int64_t k = iptr[i]; k < iptr[i + 1]; ++k) {
      int64_t c = icell[k];
      for (int64_t q = cols.ptr[c]; q < cols.ptr[c + 1]; ++q)
        if (cols.dof[q] >= 0) p.push_back(cols.dof[q]);
    }
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
  }
  for (int64_t i = 0; i < n_rows; ++i) A.rp[i + 1] = A.rp[i] + static_cast<int64_t>(pat[i].size());
  A.ci.resize(A.rp[n_rows]);
  A.v.assign(A.rp[n_rows], 0.0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n_rows; ++i) {
    const std::vector<int32_t> &p = pat[i];
    std::copy(p.begin(), p.end(), A.ci.begin() + A.rp[i]);
    double *row = A.v.data() + A.rp[i];
    for (int64_t k = iptr[i]; k < iptr[i + 1]; ++k) {
      int64_t c = icell[k];
      int32_t a = iloc[k];
      int64_t m = cols.ptr[c + 1] - cols.ptr[c];
      const double *blk = blocks.val.data() + blocks.off[c] + static_cast<int64_t>(a) * m;
      for (int64_t b = 0; b < m; ++b) {
        int32_t j = cols.dof[cols.ptr[c] + b];
        if (j < 0) continue;
        auto it = std::lower_bound(p.begin(), p.end(), j);
        row[it - p.begin()] += blk[b];
      }
    }
    std::vector<int32_t>().swap(pat[i]);
  }
  return A;
}

HostBlocks galerkin_blocks(const HostCells &fine, const HostBlocks &kf, const int32_t *parent,
                           const HostCells &coarse, const HostCSR &P) {
  const int64_t nc = coarse.n_cells;
  // children of each coarse cell, in increasing fine-cell order
  std::vector<int64_t> cptr(nc + 1, 0), child(fine.n_cells);
  for (int64_t f = 0; f < fine.n_cells; ++f) cptr[parent[f] + 1]++;
  for (int64_t c = 0; c < nc; ++c) cptr[c + 1] += cptr[c];
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t f = 0; f < fine.n_cells; ++f) child[fill[parent[f]]++] = f;
  }
  HostBlocks out;
  out.off.assign(nc + 1, 0);
  for (int64_t c = 0; c < nc; ++c) {
    int64_t m = coarse.ptr[c + 1] - coarse.ptr[c];
    out.off[c + 1] = out.off[c] + m * m;
  }
  out.val.assign(out.off[nc], 0.0);
  out.off.pop_back();
  int bad = 0;
  int64_t bad_row = -1;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
  for (int64_t E = 0; E < nc; ++E) {
    const int64_t m = coarse.ptr[E + 1] - coarse.ptr[E];
    const int32_t *cd = coarse.dof.data() + coarse.ptr[E];
    double *KE = out.val.data() + out.off[E];
    std::vector<double> Pf, T;
    for (int64_t q = cptr[E]; q < cptr[E + 1]; ++q) {
      const int64_t f = child[q];
      const int64_t nf = fine.ptr[f + 1] - fine.ptr[f];
      const int32_t *fd = fine.dof.data() + fine.ptr[f];
      Pf.assign(nf * m, 0.0);
      for (int64_t a = 0; a < nf; ++a) {
        int32_t i = fd[a];
        if (i < 0) continue;
        for (int64_t k = P.rp[i]; k < P.rp[i + 1]; ++k) {
          int32_t J = P.ci[k];
          int64_t b = 0;
          while (b < m && cd[b] != J) ++b;
          if (b == m) {
            bad = 1;
#pragma omp critical
            bad_row = i;
            continue;
          }
          Pf[a * m + b] = P.v[k];
        }
      }
      const double *Kf = kf.val.data() + kf.off[f];
      // T = K_f P_f  (nf x m), then KE += P_f^T T
      T.assign(nf * m, 0.0);
      for (int64_t a = 0; a < nf; ++a)
        for (int64_t b = 0; b < nf; ++b) {
          const double kab = Kf[a * nf + b];
          if (kab == 0.0) continue;
          const double *pb = &Pf[b * m];
          double *ta = &T[a * m];
          for (int64_t j = 0; j < m; ++j) ta[j] += kab * pb[j];
        }
      for (int64_t a = 0; a < nf; ++a) {
        const double *pa = &Pf[a * m];
        const double *ta = &T[a * m];
        for (int64_t i = 0; i < m; ++i) {
          const double w = pa[i];
          if (w == 0.0) continue;
          double *ki = KE + i * m;
          for (int64_t j = 0; j < m; ++j) ki[j] += w * ta[j];
        }
      }
    }
  }
  if (bad)
    throw SetupError{FVEM_ERR_INVALID, "prolongation row " + std::to_string(bad_row) +
                                           " references a DOF outside the parent cell (not diffusion-free)"};
  return out;
}

HostCSR transpose(const HostCSR &A) {
  HostCSR T;
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.rp.assign(T.n_rows + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) T.rp[A.ci[k] + 1]++;
  for (int64_t i = 0; i < T.n_rows; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.nnz());
  T.v.resize(A.nnz());
  std::vector<int64_t> fill(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.n_rows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t dst = fill[A.ci[k]]++;
      T.ci[dst] = static_cast<int32_t>(i);
      T.v[dst] = A.v[k];
    }
  return T;
}

std::vector<int32_t> window_order(const HostCSR &A, int64_t w) {
  const int64_t n = A.n_rows;
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < (n + w - 1) / w; ++s) {
    auto b = order.begin() + s * w, e = order.begin() + std::min(n, (s + 1) * w);
    std::stable_sort(b, e, [&](int32_t a, int32_t c) {
      return A.rp[a + 1] - A.rp[a] > A.rp[c + 1] - A.rp[c];
    });
  }
  return order;
}

HostCSR permute(const HostCSR &A, const std::vector<int32_t> &order, const std::vector<int32_t> *col_map) {
  HostCSR B;
  B.n_rows = A.n_rows;
  B.n_cols = A.n_cols;
  B.rp.assign(B.n_rows + 1, 0);
  for (int64_t r = 0; r < B.n_rows; ++r) B.rp[r + 1] = B.rp[r] + (A.rp[order[r] + 1] - A.rp[order[r]]);
  B.ci.resize(A.nnz());
  B.v.resize(A.nnz());
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < B.n_rows; ++r) {
    const int64_t o = order[r], len = A.rp[o + 1] - A.rp[o];
    std::vector<std::pair<int32_t, double>> e(len);
    for (int64_t q = 0; q < len; ++q) {
      const int32_t c = A.ci[A.rp[o] + q];
      e[q] = {col_map ? (*col_map)[c] : c, A.v[A.rp[o] + q]};
    }
    std::sort(e.begin(), e.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (int64_t q = 0; q < len; ++q) {
      B.ci[B.rp[r] + q] = e[q].first;
      B.v[B.rp[r] + q] = e[q].second;
    }
  }
  return B;
}

HostSELL to_sell(const HostCSR &A) {
  HostSELL S;
  S.n = A.n_rows;
  S.m = A.n_cols;
  S.nnz = A.nnz();
  S.nslices = (S.n + 63) / 64;
  S.sl.assign(S.nslices, 0);
  S.rl.assign(S.n, 0);
  S.sp.assign(S.nslices + 1, 0);
  for (int64_t i = 0; i < S.n; ++i) {
    S.rl[i] = static_cast<int32_t>(A.rp[i + 1] - A.rp[i]);
    S.sl[i / 64] = std::max(S.sl[i / 64], S.rl[i]);
  }
  for (int64_t s = 0; s < S.nslices; ++s) S.sp[s + 1] = S.sp[s] + 64 * static_cast<int64_t>(S.sl[s]);
  S.ci.assign(S.sp.back(), 0);
  S.v.assign(S.sp.back(), 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S.nslices; ++s)
    for (int r = 0; r < 64; ++r) {
      const int64_t i = s * 64 + r;
      const int32_t pad = static_cast<int32_t>(std::min<int64_t>(std::min(i, S.n - 1), S.m - 1));
      for (int j = 0; j < S.sl[s]; ++j) {
        const int64_t dst = S.sp[s] + 64 * static_cast<int64_t>(j) + r;
        if (i < S.n && j < S.rl[i]) {
          S.ci[dst] = A.ci[A.rp[i] + j];
          S.v[dst] = A.v[A.rp[i] + j];
        } else {
          S.ci[dst] = pad < 0 ? 0 : pad;
        }
      }
    }
  return S;
}

HostCSR from_sell(const HostSELL &S) {
  HostCSR A;
  A.n_rows = S.n;
  A.n_cols = S.m;
  A.rp.assign(S.n + 1, 0);
  for (int64_t i = 0; i < S.n; ++i) A.rp[i + 1] = A.rp[i] + S.rl[i];
  A.ci.resize(A.rp.back());
  A.v.resize(A.rp.back());
  for (int64_t i = 0; i < S.n; ++i)
    for (int j = 0; j < S.rl[i]; ++j) {
      const int64_t src = S.sp[i / 64] + 64 * static_cast<int64_t>(j) + i % 64;
      A.ci[A.rp[i] + j] = S.ci[src];
      A.v[A.rp[i] + j] = S.v[src];
    }
  return A;
}

double gershgorin_scaled(const HostCSR &A) {
  const int64_t n = A.n_rows;
  std::vector<double> dis(n, 0.0);   // 1 / sqrt(a_ii)
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i && A.v[k] > 0.0) dis[i] = 1.0 / std::sqrt(A.v[k]);
  double lmax = 0.0;
#pragma omp parallel for reduction(max : lmax)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]) * dis[A.ci[k]];
    lmax = std::max(lmax, s * dis[i]);
  }
  return lmax;
}

std::vector<int32_t> floating_components(const HostCSR &A, int32_t *n_comp) {
  const int64_t n = A.n_rows;
  std::vector<int64_t> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int64_t x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t a = find(i), b = find(A.ci[k]);
      if (a != b) parent[std::max(a, b)] = std::min(a, b);
    }
  std::vector<int64_t> root(n);
  for (int64_t i = 0; i < n; ++i) root[i] = find(i);
  // row sums relative to row magnitude, max per component
  std::vector<double> rs(n, 0.0), sc(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0, a = 0.0;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      s += A.v[k];
      a += std::fabs(A.v[k]);
    }
    rs[root[i]] = std::max(rs[root[i]], std::fabs(s));
    sc[root[i]] = std::max(sc[root[i]], a);
  }
  std::vector<int32_t> id(n, -1), comp_of_root(n, -1);
  int32_t nc = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = root[i];
    if (rs[r] > 1e-9 * sc[r]) continue;
    if (comp_of_root[r] < 0) comp_of_root[r] = nc++;
    id[i] = comp_of_root[r];
  }
  *n_comp = nc;
  return id;
}

}  // namespace fvem
