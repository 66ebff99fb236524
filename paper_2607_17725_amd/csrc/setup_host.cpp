// Host-side hierarchy setup (see setup_host.hpp).
#include "setup_host.hpp"

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>
#include <cstdio>
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
  // symbolic: sorted union of the column lists of the incident cells (its
  // length here, the list itself again in the numeric pass).  Each thread
  // marks the columns it has seen for the current row in a stamp array over
  // all columns, so only the distinct columns are sorted; the same array
  // then maps a column to its position in the row.
  auto pattern = [&](int64_t i, std::vector<int32_t> &p, std::vector<int32_t> &stamp) {
    p.clear();
    const int32_t mark = static_cast<int32_t>(i);
    for (int64_t k = iptr[i]; k < iptr[i + 1]; ++k) {
      int64_t c = icell[k];
      for (int64_t q = cols.ptr[c]; q < cols.ptr[c + 1]; ++q) {
        const int32_t j = cols.dof[q];
        if (j >= 0 && stamp[j] != mark) {
          stamp[j] = mark;
          p.push_back(j);
        }
      }
    }
    std::sort(p.begin(), p.end());
  };
#pragma omp parallel
  {
    std::vector<int32_t> p, stamp(n_cols, -1);
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n_rows; ++i) {
      pattern(i, p, stamp);
      A.rp[i + 1] = static_cast<int64_t>(p.size());
    }
  }
  for (int64_t i = 0; i < n_rows; ++i) A.rp[i + 1] += A.rp[i];
  A.ci.resize(A.rp[n_rows]);
  A.v.assign(A.rp[n_rows], 0.0);
#pragma omp parallel
  {
    std::vector<int32_t> p, stamp(n_cols, -1), pos(n_cols, 0);
    std::vector<std::pair<int32_t, double>> con;   // (entry, value) in block order
    std::vector<int32_t> start;                    // per entry: first slot of its contributions
    std::vector<double> grouped;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n_rows; ++i) {
      pattern(i, p, stamp);
      const int32_t len = static_cast<int32_t>(p.size());
      for (int32_t e = 0; e < len; ++e) pos[p[e]] = e;
      std::copy(p.begin(), p.end(), A.ci.begin() + A.rp[i]);
      double *row = A.v.data() + A.rp[i];
      // each entry sums its contributions in increasing order of value: rows
      // whose contributions coincide (translated copies of one configuration)
      // then assemble to bitwise equal values whatever the cell numbering.
      // Contributions are grouped by entry (counting sort), then each
      // entry's few values are sorted and summed.
      con.clear();
      for (int64_t k = iptr[i]; k < iptr[i + 1]; ++k) {
        int64_t c = icell[k];
        int32_t a = iloc[k];
        int64_t m = cols.ptr[c + 1] - cols.ptr[c];
        const double *blk = blocks.val.data() + blocks.off[c] + static_cast<int64_t>(a) * m;
        for (int64_t b = 0; b < m; ++b) {
          int32_t j = cols.dof[cols.ptr[c] + b];
          if (j < 0) continue;
          con.emplace_back(pos[j], blk[b]);
        }
      }
      start.assign(len + 1, 0);
      for (const auto &e : con) ++start[e.first + 1];
      for (int32_t e = 0; e < len; ++e) start[e + 1] += start[e];
      grouped.resize(con.size());
      for (const auto &e : con) grouped[start[e.first]++] = e.second;
      // start[e] is now the end of entry e's group; its begin is start[e - 1]
      int32_t b0 = 0;
      for (int32_t e = 0; e < len; ++e) {
        const int32_t b1 = start[e];
        std::sort(grouped.begin() + b0, grouped.begin() + b1);
        double acc = 0.0;
        for (int32_t t = b0; t < b1; ++t) acc += grouped[t];
        row[e] = acc;
        b0 = b1;
      }
    }
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
  // each thread owns a contiguous range of rows; per-thread column counts
  // give every (thread, column) pair its own write position, so the rows of
  // each transposed row come out in increasing order, as a serial pass would
  HostCSR T;
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  const int64_t n = A.n_rows, m = A.n_cols, nnz = A.nnz();
  const int nt = std::max(1, std::min<int>(omp_get_max_threads(), static_cast<int>((nnz >> 20) + 1)));
  std::vector<int64_t> lo(nt + 1);
  for (int t = 0; t <= nt; ++t) lo[t] = n * t / nt;
  std::vector<std::vector<int64_t>> pos(nt, std::vector<int64_t>(m, 0));
#pragma omp parallel for num_threads(nt) schedule(static, 1)
  for (int t = 0; t < nt; ++t)
    for (int64_t k = A.rp[lo[t]]; k < A.rp[lo[t + 1]]; ++k) pos[t][A.ci[k]]++;
  T.rp.assign(m + 1, 0);
  for (int64_t c = 0; c < m; ++c) {
    int64_t tot = 0;
    for (int t = 0; t < nt; ++t) tot += pos[t][c];
    T.rp[c + 1] = T.rp[c] + tot;
  }
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < m; ++c) {
    int64_t at = T.rp[c];
    for (int t = 0; t < nt; ++t) {
      const int64_t k = pos[t][c];
      pos[t][c] = at;
      at += k;
    }
  }
  T.ci.resize(nnz);
  T.v.resize(nnz);
#pragma omp parallel for num_threads(nt) schedule(static, 1)
  for (int t = 0; t < nt; ++t)
    for (int64_t i = lo[t]; i < lo[t + 1]; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int64_t dst = pos[t][A.ci[k]]++;
        T.ci[dst] = static_cast<int32_t>(i);
        T.v[dst] = A.v[k];
      }
  return T;
}

HostCSR multiply(const HostCSR &X, const HostCSR &Y) {
  HostCSR C;
  C.n_rows = X.n_rows;
  C.n_cols = Y.n_cols;
  std::vector<std::vector<int32_t>> cols(X.n_rows);
  std::vector<std::vector<double>> vals(X.n_rows);
#pragma omp parallel
  {
    std::vector<double> acc(Y.n_cols, 0.0);
    std::vector<int32_t> mark(Y.n_cols, -1), used;
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < X.n_rows; ++i) {
      used.clear();
      for (int64_t a = X.rp[i]; a < X.rp[i + 1]; ++a) {
        const int32_t k = X.ci[a];
        const double xv = X.v[a];
        for (int64_t b = Y.rp[k]; b < Y.rp[k + 1]; ++b) {
          const int32_t j = Y.ci[b];
          if (mark[j] != i) {
            mark[j] = static_cast<int32_t>(i);
            acc[j] = 0.0;
            used.push_back(j);
          }
          acc[j] += xv * Y.v[b];
        }
      }
      std::sort(used.begin(), used.end());
      cols[i] = used;
      vals[i].resize(used.size());
      for (size_t q = 0; q < used.size(); ++q) vals[i][q] = acc[used[q]];
    }
  }
  C.rp.assign(C.n_rows + 1, 0);
  for (int64_t i = 0; i < C.n_rows; ++i) C.rp[i + 1] = C.rp[i] + static_cast<int64_t>(cols[i].size());
  C.ci.resize(C.rp[C.n_rows]);
  C.v.resize(C.rp[C.n_rows]);
  for (int64_t i = 0; i < C.n_rows; ++i) {
    std::copy(cols[i].begin(), cols[i].end(), C.ci.begin() + C.rp[i]);
    std::copy(vals[i].begin(), vals[i].end(), C.v.begin() + C.rp[i]);
  }
  return C;
}

HostCSR galerkin_product(const HostCSR &A, const HostCSR &P) {
  const HostCSR AP = multiply(A, P);
  return multiply(transpose(P), AP);
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
    // full 64-row chunks (the slices) in order of their first original row,
    // so consecutive slices come from the same part of the grid
    const int64_t len = e - b, full = len / 64;
    std::vector<int64_t> ch(full);
    std::iota(ch.begin(), ch.end(), 0);
    std::vector<int32_t> first(full);
    for (int64_t c = 0; c < full; ++c) first[c] = *std::min_element(b + 64 * c, b + 64 * c + 64);
    std::stable_sort(ch.begin(), ch.end(), [&](int64_t x, int64_t y) { return first[x] < first[y]; });
    std::vector<int32_t> tmp(b, b + 64 * full);
    for (int64_t c = 0; c < full; ++c) std::copy(tmp.begin() + 64 * ch[c], tmp.begin() + 64 * ch[c] + 64, b + 64 * c);
  }
  return order;
}

HostCSR permute(const HostCSR &A, const std::vector<int32_t> &order, const std::vector<int32_t> *col_map,
                int64_t n_cols) {
  HostCSR B;
  B.n_rows = static_cast<int64_t>(order.size());
  B.n_cols = n_cols >= 0 ? n_cols : A.n_cols;
  B.rp.assign(B.n_rows + 1, 0);
  for (int64_t r = 0; r < B.n_rows; ++r)
    B.rp[r + 1] = B.rp[r] + (order[r] < 0 ? 0 : A.rp[order[r] + 1] - A.rp[order[r]]);
  B.ci.resize(B.rp[B.n_rows]);
  B.v.resize(B.rp[B.n_rows]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < B.n_rows; ++r) {
    if (order[r] < 0) continue;
    const int64_t o = order[r], len = A.rp[o + 1] - A.rp[o];
    thread_local std::vector<std::pair<int32_t, double>> e;
    e.resize(len);
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

namespace {

inline uint64_t mix64(uint64_t z) {   // SplitMix64 finaliser
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Template assignment of one value set.  quantum: relative rounding of the
// hashed values (0: exact bits); tol: accepted deviation relative to the
// row's largest entry.
void assign_templates(const HostCSR &A, const std::vector<int64_t> &ord, HostSELL &S, HostValues &V, double quantum,
                      double tol, int min_uses, int max_templates) {
  std::vector<uint64_t> key(S.n);
  std::vector<double> rmax(S.n, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < S.n; ++i) {
    double mx = 0;
    for (int64_t q = A.rp[i]; q < A.rp[i + 1]; ++q) mx = std::max(mx, std::fabs(A.v[q]));
    rmax[i] = mx;
    uint64_t h = 1469598103934665603ull ^ static_cast<uint64_t>(S.rl[i]);
    for (int64_t q = A.rp[i]; q < A.rp[i + 1]; ++q) {
      const double x = A.v[ord[q]];
      uint64_t qv;
      if (quantum > 0) {
        qv = static_cast<uint64_t>(std::llround(mx > 0 ? x / (mx * quantum) : 0.0));
      } else {
        std::memcpy(&qv, &x, sizeof qv);
      }
      h = (h ^ qv) * 1099511628211ull;
      h ^= h >> 29;
    }
    key[i] = h;
  }
  // key -> (first row, uses) in an open-addressing table; rows are visited
  // in increasing order, so the first row seen is the smallest, and the
  // table's slot a few rows ahead is fetched early
  size_t cap = 16;
  while (cap < 2 * static_cast<size_t>(S.n)) cap <<= 1;
  const uint64_t mask = cap - 1;
  std::vector<uint64_t> tkey(cap);
  std::vector<int32_t> tfirst(cap, -1), tuses(cap, 0);
  auto slot_of = [&](uint64_t k) {
    uint64_t j = mix64(k) & mask;
    while (tfirst[j] >= 0 && tkey[j] != k) j = (j + 1) & mask;
    return j;
  };
  for (int64_t i = 0; i < S.n; ++i) {
    if (i + 16 < S.n) {
      const uint64_t ja = mix64(key[i + 16]) & mask;
      __builtin_prefetch(&tkey[ja]);
      __builtin_prefetch(&tfirst[ja]);
    }
    const uint64_t j = slot_of(key[i]);
    if (tfirst[j] < 0) {
      tkey[j] = key[i];
      tfirst[j] = static_cast<int32_t>(i);
    }
    ++tuses[j];
  }
  std::vector<std::pair<int64_t, uint64_t>> popular;   // (uses, key)
  for (size_t j = 0; j < cap; ++j)
    if (tfirst[j] >= 0 && tuses[j] >= min_uses) popular.emplace_back(tuses[j], tkey[j]);
  std::sort(popular.begin(), popular.end(), [](const auto &x, const auto &y) {
    return x.first > y.first || (x.first == y.first && x.second < y.second);
  });
  if (static_cast<int>(popular.size()) > max_templates) popular.resize(max_templates);
  std::unordered_map<uint64_t, int32_t> tindex;
  std::vector<int64_t> trow;
  for (const auto &pk : popular) {
    const int64_t r = tfirst[slot_of(pk.second)];
    tindex.emplace(pk.second, V.nt++);
    trow.push_back(r);
    V.tw = std::max(V.tw, (S.rl[r] + 3) & ~3);
  }
  V.tv.assign(static_cast<size_t>(V.nt) * V.tw, 0.0);
  for (int32_t t = 0; t < V.nt; ++t) {
    const int64_t r = trow[t];
    for (int j = 0; j < S.rl[r]; ++j) V.tv[static_cast<size_t>(t) * V.tw + j] = A.v[ord[A.rp[r] + j]];
  }
  V.tid.assign(S.nslices * 64, 0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < S.n; ++i) {
    auto it = tindex.find(key[i]);
    int32_t t = -1;
    if (it != tindex.end() && S.rl[trow[it->second]] == S.rl[i]) {
      t = it->second;
      for (int j = 0; j < S.rl[i] && t >= 0; ++j)
        if (std::fabs(A.v[ord[A.rp[i] + j]] - V.tv[static_cast<size_t>(t) * V.tw + j]) > tol * rmax[i]) t = -1;
    }
    V.tid[i] = t;
  }
}

void layout_values(const HostCSR &A, const std::vector<int64_t> &ord, const HostSELL &S, HostValues &V,
                   bool templates) {
  if (!templates) {
    V.tid.assign(S.nslices * 64, 0);
    for (int64_t i = 0; i < S.n; ++i) V.tid[i] = -1;
  }
  V.vp.assign(S.nslices, -1);
  int64_t nv = 0;
  for (int64_t s = 0; s < S.nslices; ++s) {
    bool all = templates;
    for (int64_t i = s * 64; i < std::min(S.n, s * 64 + 64) && all; ++i) all = V.tid[i] >= 0;
    if (!all) {
      V.vp[s] = nv;
      nv += 64 * static_cast<int64_t>(S.sl[s]);
      for (int64_t i = s * 64; i < std::min(S.n, s * 64 + 64); ++i) V.nnz_explicit += S.rl[i];
    } else {
      V.rows_templated += std::min(S.n, s * 64 + 64) - s * 64;
    }
  }
  V.v.assign(nv, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S.nslices; ++s) {
    if (V.vp[s] < 0) continue;
    for (int r = 0; r < 64; ++r) {
      const int64_t i = s * 64 + r;
      if (i >= S.n) continue;
      for (int j = 0; j < S.rl[i]; ++j) V.v[V.vp[s] + S.at(s, j, r)] = A.v[ord[A.rp[i] + j]];
    }
  }
}

}  // namespace

HostSELL to_sell(const HostCSR &A, bool templates, int min_uses, int max_templates, bool codes) {
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
  for (int64_t s = 0; s < S.nslices; ++s) {
    S.sl[s] = (S.sl[s] + 3) & ~3;
    S.sp[s + 1] = S.sp[s] + 64 * static_cast<int64_t>(S.sl[s]);
  }
  // entry order of each row: as given, or by (value, column)
  std::vector<int64_t> ord(S.nnz);
  std::iota(ord.begin(), ord.end(), 0);
  if (templates) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < S.n; ++i)
      std::sort(ord.begin() + A.rp[i], ord.begin() + A.rp[i + 1], [&](int64_t x, int64_t y) {
        return A.v[x] < A.v[y] || (A.v[x] == A.v[y] && A.ci[x] < A.ci[y]);
      });
    assign_templates(A, ord, S, S.v64, 0.0, 0.0, min_uses, max_templates);
    assign_templates(A, ord, S, S.v32, 0x1p-30, 1e-9, min_uses, max_templates);
  }
  layout_values(A, ord, S, S.v64, templates);
  layout_values(A, ord, S, S.v32, templates);
  std::vector<int32_t> full(S.sp.back(), 0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S.nslices; ++s)
    for (int r = 0; r < 64; ++r) {
      const int64_t i = s * 64 + r;
      const int32_t pad = static_cast<int32_t>(std::min<int64_t>(std::min(i, S.n - 1), S.m - 1));
      for (int j = 0; j < S.sl[s]; ++j) {
        const bool real = i < S.n && j < S.rl[i];
        full[S.sp[s] + S.at(s, j, r)] = real ? A.ci[ord[A.rp[i] + j]] : (pad < 0 ? 0 : pad);
      }
    }
  // column codes: the distinct 1024-column blocks of each slice
  S.bt.assign(S.nslices, -1);
  S.cp.assign(S.nslices, 0);
  std::vector<std::vector<int32_t>> blocks(S.nslices);
  if (codes) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S.nslices; ++s) {
      std::vector<int32_t> &b = blocks[s];
      for (int64_t q = S.sp[s]; q < S.sp[s + 1]; ++q) b.push_back(full[q] >> 10);
      std::sort(b.begin(), b.end());
      b.erase(std::unique(b.begin(), b.end()), b.end());
      if (b.size() > 64) b.clear();
    }
  }
  int64_t n32 = 0, n16 = 0, nb = 0;
  for (int64_t s = 0; s < S.nslices; ++s) {
    const int64_t len = S.sp[s + 1] - S.sp[s];
    if (!blocks[s].empty()) {
      S.bt[s] = nb;
      nb += 64;
      S.cp[s] = n16;
      n16 += len;
    } else {
      S.cp[s] = n32;
      n32 += len;
    }
  }
  S.ci.assign(n32, 0);
  S.c16.assign(n16, 0);
  S.btab.assign(nb, 0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S.nslices; ++s) {
    const int64_t len = S.sp[s + 1] - S.sp[s];
    if (S.bt[s] < 0) {
      std::copy(full.begin() + S.sp[s], full.begin() + S.sp[s] + len, S.ci.begin() + S.cp[s]);
      continue;
    }
    const std::vector<int32_t> &b = blocks[s];
    for (size_t k = 0; k < b.size(); ++k) S.btab[S.bt[s] + k] = b[k] << 10;
    for (int64_t q = 0; q < len; ++q) {
      const int32_t c = full[S.sp[s] + q];
      const int64_t k = std::lower_bound(b.begin(), b.end(), c >> 10) - b.begin();
      S.c16[S.cp[s] + q] = static_cast<uint16_t>((k << 10) | (c & 1023));
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
  const HostValues &V = S.v64;
  for (int64_t i = 0; i < S.n; ++i) {
    const int64_t s = i / 64;
    for (int j = 0; j < S.rl[i]; ++j) {
      const int64_t off = S.at(s, j, static_cast<int>(i % 64));
      A.ci[A.rp[i] + j] = S.col(s, j, static_cast<int>(i % 64));
      A.v[A.rp[i] + j] = V.vp[s] >= 0 ? V.v[V.vp[s] + off] : V.tv[static_cast<size_t>(V.tid[i]) * V.tw + j];
    }
  }
  return A;
}

namespace {

inline uint64_t morton3(uint32_t a, uint32_t b, uint32_t c) {
  uint64_t m = 0;
  for (int i = 0; i < 21; ++i)
    m |= ((uint64_t(a >> i) & 1) << (3 * i + 2)) | ((uint64_t(b >> i) & 1) << (3 * i + 1)) |
         ((uint64_t(c >> i) & 1) << (3 * i));
  return m;
}

}  // namespace

int64_t canonical_blocks(const HostCells &C, const int32_t *lat, HostBlocks &K, double tol) {
  const int64_t nc = C.n_cells;
  // local DOFs of each aligned cell in lexicographic order of their lattice
  // offsets from the cell's lowest corner; the offsets form the group key
  std::vector<std::vector<int32_t>> perm(nc);
  std::vector<uint64_t> key(nc, 0);
  std::vector<uint8_t> aligned(nc, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t p0 = C.ptr[c], m = C.ptr[c + 1] - p0;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
    bool ok = m > 0;
    for (int64_t q = 0; q < m && ok; ++q) {
      const int32_t d = C.dof[p0 + q];
      ok = d >= 0 && lat[3 * d] >= 0;
      for (int a = 0; a < 3 && ok; ++a) lo[a] = std::min(lo[a], lat[3 * d + a]);
    }
    if (!ok) continue;
    std::vector<std::array<int32_t, 4>> rel(m);
    for (int64_t q = 0; q < m; ++q) {
      const int32_t d = C.dof[p0 + q];
      rel[q] = {lat[3 * d] - lo[0], lat[3 * d + 1] - lo[1], lat[3 * d + 2] - lo[2], static_cast<int32_t>(q)};
    }
    std::sort(rel.begin(), rel.end());
    uint64_t hsh = mix64(static_cast<uint64_t>(m));
    for (int64_t q = 0; q < m; ++q) {
      if (q > 0 && rel[q][0] == rel[q - 1][0] && rel[q][1] == rel[q - 1][1] && rel[q][2] == rel[q - 1][2]) ok = false;
      hsh = mix64(hsh ^ mix64((static_cast<uint64_t>(rel[q][0]) << 42) ^ (static_cast<uint64_t>(rel[q][1]) << 21) ^
                              static_cast<uint64_t>(rel[q][2])));
    }
    if (!ok) continue;
    perm[c].resize(m);
    for (int64_t q = 0; q < m; ++q) perm[c][q] = rel[q][3];
    key[c] = hsh;
    aligned[c] = 1;
  }
  // the first cell of each pattern (increasing cell id) is its representative
  std::unordered_map<uint64_t, int64_t> first;
  std::vector<int64_t> rep(nc, -1);
  for (int64_t c = 0; c < nc; ++c)
    if (aligned[c]) rep[c] = first.emplace(key[c], c).first->second;
  int64_t replaced = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : replaced)
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t r = rep[c];
    if (r < 0 || r == c) continue;
    const int64_t m = C.ptr[c + 1] - C.ptr[c];
    if (C.ptr[r + 1] - C.ptr[r] != m) continue;
    // same offsets (a hash collision leaves the block alone)
    bool same = true;
    for (int64_t q = 0; q < m && same; ++q) {
      const int32_t a = C.dof[C.ptr[c] + perm[c][q]], b = C.dof[C.ptr[r] + perm[r][q]];
      for (int x = 0; x < 3; ++x)
        same = same && lat[3 * a + x] - lat[3 * C.dof[C.ptr[c] + perm[c][0]] + x] ==
                           lat[3 * b + x] - lat[3 * C.dof[C.ptr[r] + perm[r][0]] + x];
    }
    if (!same) continue;
    const double *Br = &K.val[K.off[r]];
    double *Bc = &K.val[K.off[c]];
    double big = 0, diff = 0;
    for (int64_t i = 0; i < m * m; ++i) big = std::max(big, std::fabs(Br[i]));
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < m; ++j)
        diff = std::max(diff, std::fabs(Bc[perm[c][i] * m + perm[c][j]] - Br[perm[r][i] * m + perm[r][j]]));
    if (diff > tol * big) continue;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < m; ++j) Bc[perm[c][i] * m + perm[c][j]] = Br[perm[r][i] * m + perm[r][j]];
    ++replaced;
  }
  return replaced;
}

bool lattice_layout(const HostCSR &A, const int32_t *lat, int32_t lat_n, double min_fraction, HostLattice *L) {
  *L = HostLattice();
  const int64_t n = A.n_rows;
  if (!lat || lat_n < 3 || n == 0) return false;
  const int64_t ln = lat_n, ln3 = ln * ln * ln;
  // point -> DOF; a point claimed twice leaves the lattice for both DOFs
  std::vector<int32_t> pt(ln3, -1);
  std::vector<uint8_t> on(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t a = lat[3 * i], b = lat[3 * i + 1], c = lat[3 * i + 2];
    if (a < 0 || b < 0 || c < 0 || a >= lat_n || b >= lat_n || c >= lat_n) continue;
    int32_t &q = pt[(a * ln + b) * ln + c];
    if (q == -1) {
      q = static_cast<int32_t>(i);
      on[i] = 1;
    } else {
      if (q >= 0) on[q] = 0;
      q = -2;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (on[i] && pt[(lat[3 * i] * ln + lat[3 * i + 1]) * ln + lat[3 * i + 2]] != i) on[i] = 0;
  auto cls = [&](int64_t i) { return 4 * (lat[3 * i] & 1) + 2 * (lat[3 * i + 1] & 1) + (lat[3 * i + 2] & 1); };
  // dense stencil of a row in offset space; false if some column is off the lattice or too far
  auto dense = [&](int64_t i, double *v, uint8_t *p) {
    std::fill(p, p + STENCIL_MAX, 0);
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t j = A.ci[k];
      if (!on[j]) return false;
      const int da = lat[3 * j] - lat[3 * i], db = lat[3 * j + 1] - lat[3 * i + 1], dc = lat[3 * j + 2] - lat[3 * i + 2];
      if (da < -2 || da > 2 || db < -2 || db > 2 || dc < -2 || dc > 2) return false;
      const int code = (da + 2) * 25 + (db + 2) * 5 + (dc + 2);
      v[code] = A.v[k];
      p[code] = 1;
    }
    return true;
  };
  auto hash = [&](const double *v, const uint8_t *p) {
    uint64_t hsh = 0x12345;
    for (int q = 0; q < STENCIL_MAX; ++q)
      if (p[q]) {
        uint64_t bits;
        std::memcpy(&bits, &v[q], 8);
        hsh = mix64(hsh ^ (static_cast<uint64_t>(q) << 56) ^ mix64(bits));
      }
    return hsh;
  };
  std::vector<uint64_t> rh(n, 0);
  std::vector<uint8_t> elig(n, 0);
#pragma omp parallel
  {
    double v[STENCIL_MAX];
    uint8_t p[STENCIL_MAX];
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      if (!on[i] || !dense(i, v, p)) continue;
      elig[i] = 1;
      rh[i] = hash(v, p);
    }
  }
  // reference stencil of each class: its most frequent row (at least 64 rows)
  int64_t ref_row[8];
  for (int t = 0; t < 8; ++t) {
    std::unordered_map<uint64_t, std::pair<int64_t, int64_t>> cnt;   // hash -> (count, first row)
    for (int64_t i = 0; i < n; ++i)
      if (elig[i] && cls(i) == t) {
        auto it = cnt.find(rh[i]);
        if (it == cnt.end()) cnt.emplace(rh[i], std::make_pair(int64_t(1), i));
        else ++it->second.first;
      }
    ref_row[t] = -1;
    int64_t best = 63;
    for (const auto &kv : cnt)
      if (kv.second.first > best || (kv.second.first == best && ref_row[t] >= 0 && kv.second.second < ref_row[t])) {
        best = kv.second.first;
        ref_row[t] = kv.second.second;
      }
  }
  std::vector<double> rv(8 * STENCIL_MAX, 0.0);
  std::vector<uint8_t> rp(8 * STENCIL_MAX, 0);
  for (int t = 0; t < 8; ++t)
    if (ref_row[t] >= 0) dense(ref_row[t], &rv[STENCIL_MAX * t], &rp[STENCIL_MAX * t]);
  L->is_stencil.assign(n, 0);
  int64_t nst = 0, nnzst = 0;
#pragma omp parallel
  {
    double v[STENCIL_MAX];
    uint8_t p[STENCIL_MAX];
#pragma omp for schedule(dynamic, 4096) reduction(+ : nst, nnzst)
    for (int64_t i = 0; i < n; ++i) {
      if (!elig[i]) continue;
      const int t = cls(i);
      if (ref_row[t] < 0 || rh[i] != rh[ref_row[t]]) continue;
      dense(i, v, p);
      bool same = true;
      for (int q = 0; q < STENCIL_MAX && same; ++q)
        same = p[q] == rp[STENCIL_MAX * t + q] && (!p[q] || std::memcmp(&v[q], &rv[STENCIL_MAX * t + q], 8) == 0);
      if (!same) continue;
      L->is_stencil[i] = 1;
      ++nst;
      nnzst += A.rp[i + 1] - A.rp[i];
    }
  }
  if (static_cast<double>(nst) < min_fraction * static_cast<double>(n)) {
    *L = HostLattice();
    return false;
  }
  L->n_stencil = nst;
  L->nnz_stencil = nnzst;
  L->lat_n = lat_n;
  const int32_t tn = (lat_n + 7) / 8;
  L->tn = tn;
  const int64_t tn3 = static_cast<int64_t>(tn) * tn * tn;
  // tiles holding a lattice DOF, in Morton order
  std::vector<uint8_t> used(tn3, 0);
  for (int64_t i = 0; i < n; ++i)
    if (on[i]) used[((lat[3 * i] >> 3) * tn + (lat[3 * i + 1] >> 3)) * tn + (lat[3 * i + 2] >> 3)] = 1;
  std::vector<std::pair<uint64_t, int32_t>> mt;
  for (int64_t t = 0; t < tn3; ++t)
    if (used[t]) mt.emplace_back(morton3(t / (tn * tn), (t / tn) % tn, t % tn), static_cast<int32_t>(t));
  std::sort(mt.begin(), mt.end());
  L->tile_base.assign(tn3, -1);
  for (size_t r = 0; r < mt.size(); ++r) L->tile_base[mt[r].second] = static_cast<int32_t>(512 * r);
  const int64_t nslot = 512 * static_cast<int64_t>(mt.size());
  if (nslot + n >= (int64_t(1) << 31)) {
    *L = HostLattice();
    return false;
  }
  L->order.assign(nslot, -1);
  std::vector<uint64_t> tmask(8 * mt.size(), 0);
  for (int64_t i = 0; i < n; ++i) {
    if (!on[i]) continue;
    const int a = lat[3 * i], b = lat[3 * i + 1], c = lat[3 * i + 2];
    const int64_t tile = ((a >> 3) * tn + (b >> 3)) * tn + (c >> 3);
    const int t = cls(i);
    const int pos = 16 * ((a & 7) >> 1) + 4 * ((b & 7) >> 1) + ((c & 7) >> 1);
    const int64_t slot = L->tile_base[tile] + 64 * t + pos;
    L->order[slot] = static_cast<int32_t>(i);
    if (L->is_stencil[i]) tmask[8 * (L->tile_base[tile] / 512) + t] |= uint64_t(1) << pos;
  }
  for (int64_t i = 0; i < n; ++i)
    if (!on[i]) L->order.push_back(static_cast<int32_t>(i));
  for (size_t r = 0; r < mt.size(); ++r) {
    bool any = false;
    for (int t = 0; t < 8; ++t) any = any || tmask[8 * r + t];
    if (!any) continue;
    L->tiles.push_back(mt[r].second);
    for (int t = 0; t < 8; ++t) L->mask.push_back(tmask[8 * r + t]);
  }
  // class tables: entries in increasing offset code; LDS offsets into the
  // class-major 6x6x6 halo of the neighbour's class
  L->off.assign(8 * 128, 0);
  L->delta.assign(8 * 128, 0);
  L->val.assign(8 * 128, 0.0);
  for (int t = 0; t < 8; ++t) {
    int m = 0;
    const int ta = t >> 2, tb = (t >> 1) & 1, tc = t & 1;
    for (int q = 0; q < STENCIL_MAX; ++q) {
      if (!rp[STENCIL_MAX * t + q]) continue;
      const int da = q / 25 - 2, db = (q / 5) % 5 - 2, dc = q % 5 - 2;
      const int ua = (ta + da) & 1, ub = (tb + db) & 1, uc = (tc + dc) & 1;
      const int ea = (ta + da + 2 - ua) / 2, eb = (tb + db + 2 - ub) / 2, ec = (tc + dc + 2 - uc) / 2;
      L->off[128 * t + m] = (4 * ua + 2 * ub + uc) * STENCIL_SUB + ea * STENCIL_P1 + eb * STENCIL_P2 + ec;
      L->delta[128 * t + m] = q;
      L->val[128 * t + m] = rv[STENCIL_MAX * t + q];
      ++m;
    }
    L->len[t] = m;
  }
  return true;
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
