// Checks of the library's host-side setup routines (sliced storage, level
// order, permutation, transpose, block assembly, element-wise Galerkin
// product, scaled Gershgorin bound, canonical element blocks) against dense
// brute force on small random inputs, or against hand-built cases.  Built
// with g++ by tests/test_host_setup.py; prints one line per check and exits
// non-zero on the first failure.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2607_17725_amd/csrc/setup_host.hpp"

using namespace fvem;

static int failures = 0;

static void expect(bool ok, const char *what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++failures;
}

static std::vector<double> dense(const HostCSR &A) {
  std::vector<double> D(A.n_rows * A.n_cols, 0.0);
  for (int64_t i = 0; i < A.n_rows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) D[i * A.n_cols + A.ci[k]] += A.v[k];
  return D;
}

static HostCSR random_csr(std::mt19937 &g, int64_t n, int64_t m, int maxlen) {
  std::uniform_int_distribution<int> len(0, maxlen), col(0, static_cast<int>(m - 1));
  std::normal_distribution<double> val;
  HostCSR A;
  A.n_rows = n;
  A.n_cols = m;
  A.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int> c;
    const int l = len(g);
    for (int q = 0; q < l; ++q) {
      const int j = col(g);
      bool dup = false;
      for (int x : c) dup = dup || x == j;
      if (!dup) c.push_back(j);
    }
    for (int j : c) {
      A.ci.push_back(j);
      A.v.push_back(val(g));
    }
    A.rp[i + 1] = static_cast<int64_t>(A.ci.size());
  }
  return A;
}

static double maxdiff(const std::vector<double> &a, const std::vector<double> &b) {
  double d = a.size() == b.size() ? 0.0 : INFINITY;
  for (size_t i = 0; i < a.size() && i < b.size(); ++i) d = std::max(d, std::fabs(a[i] - b[i]));
  return d;
}

int main() {
  std::mt19937 g(7);
  // sliced storage round trip, ragged last slice and empty rows
  for (int64_t n : {1, 63, 64, 65, 200, 1000}) {
    HostCSR A = random_csr(g, n, n + 3, 90);
    HostSELL S = to_sell(A);
    bool ok = S.nslices == (n + 63) / 64 && S.sp.back() % 64 == 0;
    for (int64_t s = 0; s < S.nslices; ++s) {
      int mx = 0;
      for (int64_t i = s * 64; i < std::min(n, s * 64 + 64); ++i) mx = std::max<int>(mx, static_cast<int>(A.rp[i + 1] - A.rp[i]));
      ok = ok && S.sl[s] == ((mx + 3) & ~3);
    }
    for (int32_t c : S.ci) ok = ok && c >= 0 && c < A.n_cols;
    ok = ok && S.c16.empty();
    // padding contributes zero: a dense product through the slices equals A x
    std::vector<double> x(A.n_cols), y(n, 0.0);
    for (auto &v : x) v = std::normal_distribution<double>()(g);
    for (int64_t s = 0; s < S.nslices; ++s)
      for (int r = 0; r < 64; ++r) {
        const int64_t i = s * 64 + r;
        if (i >= n) continue;
        for (int j = 0; j < S.sl[s]; ++j)
          y[i] += S.v64.v[S.v64.vp[s] + S.at(s, j, r)] * x[S.col(s, j, r)];
      }
    std::vector<double> yr(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) yr[i] += A.v[k] * x[A.ci[k]];
    ok = ok && maxdiff(y, yr) < 1e-12;
    const HostCSR B = from_sell(S);
    ok = ok && B.rp == A.rp && B.ci == A.ci && B.v == A.v;
    char msg[96];
    std::snprintf(msg, sizeof msg, "sliced storage round trip, n=%lld", static_cast<long long>(n));
    expect(ok, msg);
  }
  // column codes on random rows: narrow column ranges code, wide ones do not
  for (int64_t m : {3000, 400000}) {
    HostCSR A = random_csr(g, 300, m, 70);
    HostSELL S = to_sell(A, false, 64, 1024, true);
    int coded = 0;
    for (int64_t s2 = 0; s2 < S.nslices; ++s2) coded += S.bt[s2] >= 0;
    const HostCSR B = from_sell(S);
    char msg[96];
    std::snprintf(msg, sizeof msg, "column codes round trip, %lld columns (%d of %lld slices coded)",
                  static_cast<long long>(m), coded, static_cast<long long>(S.nslices));
    expect(B.rp == A.rp && B.ci == A.ci && B.v == A.v && (m == 3000 ? coded == S.nslices : coded == 0), msg);
  }
  // value templates: a 7-point stencil on a 3-D grid (translation-invariant
  // interior rows, boundary rows differ) plus perturbed rows
  {
    const int gs = 12, n = gs * gs * gs;
    HostCSR A;
    A.n_rows = A.n_cols = n;
    A.rp.assign(n + 1, 0);
    std::mt19937 gg(3);
    std::uniform_int_distribution<int> pick(0, n - 1);
    std::vector<int> noisy(n, 0);
    for (int q = 0; q < 8; ++q) noisy[pick(gg)] = 1;
    for (int i = 0; i < n; ++i) {
      const int x = i % gs, y = (i / gs) % gs, z = i / (gs * gs);
      const int nb[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
      std::vector<std::pair<int, double>> e{{i, 6.5}};
      for (int k = 0; k < 6; ++k) {
        const int X = x + nb[k][0], Y = y + nb[k][1], Z = z + nb[k][2];
        if (X < 0 || Y < 0 || Z < 0 || X >= gs || Y >= gs || Z >= gs) continue;
        e.push_back({(Z * gs + Y) * gs + X, -1.0 - 0.1 * k});
      }
      std::sort(e.begin(), e.end());
      for (auto &pr : e) {
        A.ci.push_back(pr.first);
        A.v.push_back(pr.second + (noisy[i] ? 1e-3 * pr.first : 0.0) + (pr.first == i ? 1e-15 * (i % 3) : 0.0));
      }
      A.rp[i + 1] = static_cast<int64_t>(A.ci.size());
    }
    HostSELL S = to_sell(A, true, 4, 1024, true);
    {
      // columns through the codes: the coded slices decode to what the
      // uncoded storage holds
      const HostSELL U = to_sell(A, true, 4, 1024, false);
      int coded = 0;
      bool same = true;
      for (int64_t s2 = 0; s2 < S.nslices; ++s2) {
        coded += S.bt[s2] >= 0;
        for (int r = 0; r < 64; ++r)
          for (int j = 0; j < S.sl[s2]; ++j) same = same && S.col(s2, j, r) == U.col(s2, j, r);
      }
      char m2[96];
      std::snprintf(m2, sizeof m2, "16-bit column codes (%d of %lld slices coded)", coded,
                    static_cast<long long>(S.nslices));
      expect(same && coded > 0, m2);
    }
    std::vector<double> x(n);
    for (auto &v : x) v = std::normal_distribution<double>()(gg);
    std::vector<double> yr(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) yr[i] += A.v[k] * x[A.ci[k]];
    double ymax = 0;
    for (double v : yr) ymax = std::max(ymax, std::fabs(v));
    for (int set = 0; set < 2; ++set) {
      const HostValues &V = set == 0 ? S.v64 : S.v32;
      int templated_slices = 0;
      for (int64_t s2 = 0; s2 < S.nslices; ++s2) templated_slices += V.vp[s2] < 0;
      std::vector<double> y(n, 0.0);
      for (int64_t s2 = 0; s2 < S.nslices; ++s2)
        for (int r = 0; r < 64; ++r) {
          const int64_t i = s2 * 64 + r;
          if (i >= n) continue;
          for (int j = 0; j < S.sl[s2]; ++j) {
            const double v = V.vp[s2] >= 0 ? V.v[V.vp[s2] + S.at(s2, j, r)] : V.tv[static_cast<size_t>(V.tid[i]) * V.tw + j];
            y[i] += v * x[S.col(s2, j, r)];
          }
        }
      // FP64 templates are exact: the diagonal's 1e-15 jitter splits them;
      // the single-precision set absorbs it
      const double tol = set == 0 ? 1e-14 : 1e-9;
      char msg[160];
      std::snprintf(msg, sizeof msg, "value templates (%s): %d templates, %d of %lld slices without values",
                    set == 0 ? "exact" : "single", V.nt, templated_slices, static_cast<long long>(S.nslices));
      expect(V.nt >= 4 && templated_slices >= 2 && maxdiff(y, yr) < tol * ymax && V.tw % 4 == 0, msg);
      bool noisy_ok = true;
      for (int i = 0; i < n; ++i) noisy_ok = noisy_ok && (!noisy[i] || V.tid[i] < 0);
      expect(noisy_ok, "rows that differ from every template store their values");
      bool exact_ok = true;
      if (set == 0)
        for (int i = 0; i < n; ++i)
          if (V.tid[i] >= 0) {
            std::vector<double> rowv(A.v.begin() + A.rp[i], A.v.begin() + A.rp[i + 1]);
            std::sort(rowv.begin(), rowv.end());
            for (size_t j = 0; j < rowv.size(); ++j) exact_ok = exact_ok && rowv[j] == V.tv[static_cast<size_t>(V.tid[i]) * V.tw + j];
          }
      if (set == 0) expect(exact_ok, "exact templates reproduce their rows bitwise");
    }
    const HostCSR B = from_sell(S);
    expect(maxdiff(dense(B), dense(A)) == 0.0, "read-back of the exact value set");
  }
  // level order: a permutation that keeps every window's rows, sorts each
  // 64-row chunk by decreasing length (stable) and orders a window's full
  // chunks by their smallest original row
  {
    HostCSR A = random_csr(g, 1000, 1000, 40);
    const int64_t w = 256;
    std::vector<int32_t> o = window_order(A, w);
    std::vector<int> seen(1000, 0);
    bool ok = o.size() == 1000;
    for (int32_t i : o) ok = ok && i >= 0 && i < 1000 && !seen[i]++;
    for (int64_t r = 0; r < 1000; ++r) ok = ok && o[r] / w == r / w;
    // rows of the window sorted by (decreasing length, index), cut into chunks
    for (int64_t s0 = 0; s0 < 1000; s0 += w) {
      const int64_t e0 = std::min<int64_t>(1000, s0 + w);
      std::vector<int32_t> ref(e0 - s0);
      for (int64_t r = s0; r < e0; ++r) ref[r - s0] = static_cast<int32_t>(r);
      std::stable_sort(ref.begin(), ref.end(), [&](int32_t a, int32_t c) {
        return A.rp[a + 1] - A.rp[a] > A.rp[c + 1] - A.rp[c];
      });
      const int64_t full = (e0 - s0) / 64;
      std::vector<std::vector<int32_t>> chunks;
      for (int64_t c = 0; c < full; ++c) chunks.emplace_back(ref.begin() + 64 * c, ref.begin() + 64 * c + 64);
      std::stable_sort(chunks.begin(), chunks.end(), [](const auto &x, const auto &y) {
        return *std::min_element(x.begin(), x.end()) < *std::min_element(y.begin(), y.end());
      });
      std::vector<int32_t> expect_o;
      for (auto &c : chunks) expect_o.insert(expect_o.end(), c.begin(), c.end());
      expect_o.insert(expect_o.end(), ref.begin() + 64 * full, ref.end());
      for (int64_t r = s0; r < e0; ++r) ok = ok && o[r] == expect_o[r - s0];
    }
    expect(ok, "window order");
    // symmetric renumbering: B = Q A Q^T with columns sorted per row
    std::vector<int32_t> inv(1000);
    for (int i = 0; i < 1000; ++i) inv[o[i]] = i;
    HostCSR B = permute(A, o, &inv);
    const std::vector<double> DA = dense(A), DB = dense(B);
    bool same = true, sorted = true;
    for (int64_t r = 0; r < 1000; ++r)
      for (int64_t c = 0; c < 1000; ++c) same = same && DB[r * 1000 + c] == DA[o[r] * 1000 + o[c]];
    for (int64_t r = 0; r < 1000; ++r)
      for (int64_t k = B.rp[r]; k + 1 < B.rp[r + 1]; ++k) sorted = sorted && B.ci[k] < B.ci[k + 1];
    expect(same && sorted, "symmetric renumbering");
    HostCSR C = permute(B, inv, &o);
    expect(dense(C) == DA, "renumbering inverts");
  }
  // transpose
  {
    HostCSR A = random_csr(g, 300, 170, 30);
    HostCSR T = transpose(A);
    const std::vector<double> DA = dense(A), DT = dense(T);
    bool ok = T.n_rows == 170 && T.n_cols == 300;
    for (int64_t i = 0; i < 300; ++i)
      for (int64_t j = 0; j < 170; ++j) ok = ok && DA[i * 170 + j] == DT[j * 300 + i];
    expect(ok, "transpose");
  }
  // multithreaded transpose (several million nonzeros) against a serial
  // counting-sort transpose: same arrays, rows ascending in every column
  {
    HostCSR A = random_csr(g, 200000, 50000, 40);
    HostCSR T = transpose(A);
    HostCSR R;
    R.n_rows = A.n_cols;
    R.n_cols = A.n_rows;
    R.rp.assign(R.n_rows + 1, 0);
    for (int64_t k = 0; k < A.nnz(); ++k) R.rp[A.ci[k] + 1]++;
    for (int64_t c = 0; c < R.n_rows; ++c) R.rp[c + 1] += R.rp[c];
    R.ci.resize(A.nnz());
    R.v.resize(A.nnz());
    std::vector<int64_t> fill(R.rp.begin(), R.rp.end() - 1);
    for (int64_t i = 0; i < A.n_rows; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        R.ci[fill[A.ci[k]]] = static_cast<int32_t>(i);
        R.v[fill[A.ci[k]]++] = A.v[k];
      }
    char msg[96];
    std::snprintf(msg, sizeof msg, "transpose of %lld nonzeros matches the serial one",
                  static_cast<long long>(A.nnz()));
    expect(T.rp == R.rp && T.ci == R.ci && T.v == R.v, msg);
  }
  // block assembly and element-wise Galerkin product against dense sums
  {
    const int nf = 40, nc = 12, ncell_f = 18, ncell_c = 4, mf = 6, mc = 5;
    std::uniform_int_distribution<int> df(-1, nf - 1), dc(0, nc - 1);
    HostCells F, Cc;
    F.n_cells = ncell_f;
    Cc.n_cells = ncell_c;
    F.ptr.push_back(0);
    Cc.ptr.push_back(0);
    std::vector<int32_t> parent(ncell_f);
    for (int c = 0; c < ncell_c; ++c) {
      std::vector<int> d;
      while (static_cast<int>(d.size()) < mc) {
        int j = dc(g);
        bool dup = false;
        for (int x : d) dup = dup || x == j;
        if (!dup) d.push_back(j);
      }
      for (int j : d) Cc.dof.push_back(j);
      Cc.ptr.push_back(static_cast<int64_t>(Cc.dof.size()));
    }
    for (int c = 0; c < ncell_f; ++c) {
      std::vector<int> d;
      while (static_cast<int>(d.size()) < mf) {
        int j = df(g);
        bool dup = false;
        for (int x : d) dup = dup || (x == j && j >= 0);
        if (!dup) d.push_back(j);
      }
      for (int j : d) F.dof.push_back(j);
      F.ptr.push_back(static_cast<int64_t>(F.dof.size()));
      parent[c] = c % ncell_c;
    }
    HostBlocks K;
    K.off.resize(ncell_f);
    for (int c = 0; c < ncell_f; ++c) {
      K.off[c] = static_cast<int64_t>(K.val.size());
      std::vector<double> M(mf * mf);
      for (auto &v : M) v = std::normal_distribution<double>()(g);
      for (int a = 0; a < mf; ++a)
        for (int b = 0; b < mf; ++b) K.val.push_back(M[a * mf + b] + M[b * mf + a]);
    }
    HostCSR A = assemble_blocks(nf, nf, F, F, K);
    std::vector<double> DA(nf * nf, 0.0);
    for (int c = 0; c < ncell_f; ++c)
      for (int a = 0; a < mf; ++a)
        for (int b = 0; b < mf; ++b) {
          const int i = F.dof[F.ptr[c] + a], j = F.dof[F.ptr[c] + b];
          if (i >= 0 && j >= 0) DA[i * nf + j] += K.val[K.off[c] + a * mf + b];
        }
    expect(maxdiff(dense(A), DA) < 1e-12, "block assembly");
    // a prolongation whose rows only reach the coarse DOFs of every parent
    // of the cells holding the fine DOF
    std::vector<std::vector<int>> allowed(nf);
    for (int c = 0; c < ncell_f; ++c)
      for (int a = 0; a < mf; ++a) {
        const int i = F.dof[F.ptr[c] + a];
        if (i < 0) continue;
        std::vector<int> here(Cc.dof.begin() + Cc.ptr[parent[c]], Cc.dof.begin() + Cc.ptr[parent[c] + 1]);
        if (allowed[i].empty()) {
          allowed[i] = here;
          allowed[i].push_back(-2);   // marks "initialised"
        } else {
          std::vector<int> keep{-2};
          for (int j : allowed[i])
            for (int q : here)
              if (j == q) keep.push_back(j);
          allowed[i] = keep;
        }
      }
    HostCSR P;
    P.n_rows = nf;
    P.n_cols = nc;
    P.rp.assign(nf + 1, 0);
    for (int i = 0; i < nf; ++i) {
      for (int j : allowed[i])
        if (j >= 0 && std::uniform_real_distribution<double>()(g) < 0.7) {
          P.ci.push_back(j);
          P.v.push_back(std::normal_distribution<double>()(g));
        }
      P.rp[i + 1] = static_cast<int64_t>(P.ci.size());
    }
    HostBlocks Kc = galerkin_blocks(F, K, parent.data(), Cc, P);
    HostCSR Ac = assemble_blocks(nc, nc, Cc, Cc, Kc);
    const std::vector<double> DP = dense(P);
    std::vector<double> R(nc * nc, 0.0);
    for (int a = 0; a < nc; ++a)
      for (int b = 0; b < nc; ++b)
        for (int i = 0; i < nf; ++i)
          for (int j = 0; j < nf; ++j) R[a * nc + b] += DP[i * nc + a] * DA[i * nf + j] * DP[j * nc + b];
    double scale = 0.0;
    for (double v : R) scale = std::max(scale, std::fabs(v));
    expect(maxdiff(dense(Ac), R) < 1e-12 * scale, "element-wise Galerkin product equals P^T A P");
  }
  // scaled Gershgorin bound of D^-1/2 A D^-1/2 for the 1D Laplacian: 2
  {
    const int n = 50;
    HostCSR A;
    A.n_rows = A.n_cols = n;
    A.rp.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      for (int j = i - 1; j <= i + 1; ++j)
        if (j >= 0 && j < n) {
          A.ci.push_back(j);
          A.v.push_back(j == i ? 4.0 : -2.0);
        }
      A.rp[i + 1] = static_cast<int64_t>(A.ci.size());
    }
    expect(std::fabs(gershgorin_scaled(A) - 2.0) < 1e-14, "scaled Gershgorin bound");
  }
  {
    // canonical blocks: four 2-DOF cells on a 1D lattice (x along the first
    // coordinate), each cell's DOFs at x and x+1 but listed in either order;
    // cell 1 is cell 0 translated with a 1e-15 perturbation, cell 2 differs
    // by 1e-9, cell 3 has a different pattern (DOFs two apart), cell 4 has a
    // DOF off the lattice
    HostCells C;
    C.n_cells = 5;
    C.ptr = {0, 2, 4, 6, 8, 10};
    C.dof = {0, 1, 3, 2, 4, 5, 6, 8, 9, 10};
    std::vector<int32_t> lat = {0, 0, 0, 1, 0, 0, 2, 0, 0, 3, 0, 0, 4, 0, 0, 5, 0, 0,
                                6, 0, 0, 7, 0, 0, 8, 0, 0, -1, -1, -1, 9, 0, 0};
    HostBlocks K;
    K.off = {0, 4, 8, 12, 16};
    // cell 0 in order (x, x+1); cell 1 lists (x+1, x): its block is the
    // transpose-permuted copy
    K.val = {4.0, -1.0, -1.0, 2.0,
             2.0, -1.0 + 1e-15, -1.0, 4.0,
             4.0, -1.0 + 1e-9, -1.0, 2.0,
             4.0, -1.0, -1.0, 2.0,
             4.0, -1.0, -1.0, 2.0};
    const int64_t n = canonical_blocks(C, lat.data(), K, 1e-12);
    expect(n == 1, "canonical blocks: one translated copy replaced");
    expect(K.val[4] == 2.0 && K.val[5] == -1.0 && K.val[6] == -1.0 && K.val[7] == 4.0,
           "canonical blocks: the copy takes the first block in its own local order");
    expect(K.val[9] == -1.0 + 1e-9, "canonical blocks: a block beyond the tolerance is kept");
  }
  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
