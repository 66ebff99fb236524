// Check of the lattice stencil layout (lattice_layout in setup_host.cpp) on
// an operator read from files: the padded order holds every DOF once, the
// masks flag exactly the stencil rows, and an emulation of the stencil
// kernel's addressing (tile slots, class-major halo sub-grids, table
// offsets) reproduces A x on every stencil row.  Built with g++ by
// tests/test_lattice_layout.py; exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2607_17725_amd/csrc/setup_host.hpp"

using namespace fvem;

template <typename T>
static std::vector<T> read_file(const char *path) {
  std::FILE *f = std::fopen(path, "rb");
  if (!f) {
    std::printf("FAIL cannot open %s\n", path);
    std::exit(2);
  }
  std::fseek(f, 0, SEEK_END);
  const long bytes = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  std::vector<T> v(bytes / sizeof(T));
  if (!v.empty() && std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) std::exit(2);
  std::fclose(f);
  return v;
}

static int fail(const char *what) {
  std::printf("FAIL %s\n", what);
  return 1;
}

int main(int argc, char **argv) {
  if (argc != 7) return fail("usage: rp ci val lat lat_n min_stencil_fraction");
  HostCSR A;
  A.rp = read_file<int64_t>(argv[1]);
  A.ci = read_file<int32_t>(argv[2]);
  A.v = read_file<double>(argv[3]);
  A.n_rows = A.n_cols = static_cast<int64_t>(A.rp.size()) - 1;
  const std::vector<int32_t> lat = read_file<int32_t>(argv[4]);
  const int32_t lat_n = std::atoi(argv[5]);
  const double want = std::atof(argv[6]);
  const int64_t n = A.n_rows;
  HostLattice L;
  if (!lattice_layout(A, lat.data(), lat_n, 0.0, &L)) return fail("layout refused");
  std::printf("rows %lld stencil rows %lld (%.3f) tiles %zu classes", static_cast<long long>(n),
              static_cast<long long>(L.n_stencil), double(L.n_stencil) / n, L.tiles.size());
  for (int t = 0; t < 8; ++t) std::printf(" %d", L.len[t]);
  std::printf("\n");
  if (double(L.n_stencil) < want * n) return fail("too few stencil rows");
  // every DOF exactly once in the padded order
  std::vector<int> seen(n, 0);
  for (int32_t i : L.order) {
    if (i < -1 || i >= n) return fail("order entry out of range");
    if (i >= 0) ++seen[i];
  }
  for (int64_t i = 0; i < n; ++i)
    if (seen[i] != 1) return fail("DOF not exactly once in the order");
  std::vector<int64_t> slot(n, -1);
  for (size_t r = 0; r < L.order.size(); ++r)
    if (L.order[r] >= 0) slot[L.order[r]] = static_cast<int64_t>(r);
  // masks agree with is_stencil
  int64_t flagged = 0;
  const int tn = L.tn;
  for (size_t b = 0; b < L.tiles.size(); ++b)
    for (int t = 0; t < 8; ++t)
      for (int lane = 0; lane < 64; ++lane) {
        if (!((L.mask[8 * b + t] >> lane) & 1)) continue;
        ++flagged;
        const int32_t i = L.order[L.tile_base[L.tiles[b]] + 64 * t + lane];
        if (i < 0 || !L.is_stencil[i]) return fail("mask flags a slot without a stencil row");
      }
  if (flagged != L.n_stencil) return fail("mask count differs from the stencil row count");
  // emulate the kernel on a random x in the padded layout
  std::mt19937 gen(5);
  std::normal_distribution<double> nd;
  std::vector<double> xc(n), xp(L.order.size() + 1, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    xc[i] = nd(gen);
    xp[slot[i]] = xc[i];
  }
  std::vector<double> halo(8 * STENCIL_SUB);
  double worst = 0.0;
  for (size_t b = 0; b < L.tiles.size(); ++b) {
    const int32_t tile = L.tiles[b];
    const int Ta = tile / (tn * tn), Tb = (tile / tn) % tn, Tc = tile % tn;
    std::fill(halo.begin(), halo.end(), 0.0);
    for (int e = 0; e < 1728; ++e) {
      const int tp = e / 216, r = e % 216, I = r / 36, J = (r / 6) % 6, K = r % 6;
      const int a = 8 * Ta - 2 + (tp >> 2) + 2 * I, bb = 8 * Tb - 2 + ((tp >> 1) & 1) + 2 * J,
                c = 8 * Tc - 2 + (tp & 1) + 2 * K;
      double v = 0.0;
      if (a >= 0 && a < lat_n && bb >= 0 && bb < lat_n && c >= 0 && c < lat_n) {
        const int32_t base = L.tile_base[((a >> 3) * tn + (bb >> 3)) * tn + (c >> 3)];
        if (base >= 0) v = xp[base + 64 * tp + 16 * ((a & 7) >> 1) + 4 * ((bb & 7) >> 1) + ((c & 7) >> 1)];
      }
      halo[tp * STENCIL_SUB + I * STENCIL_P1 + J * STENCIL_P2 + K] = v;
    }
    for (int t = 0; t < 8; ++t)
      for (int lane = 0; lane < 64; ++lane) {
        if (!((L.mask[8 * b + t] >> lane) & 1)) continue;
        const int hp = (lane >> 4) * STENCIL_P1 + ((lane >> 2) & 3) * STENCIL_P2 + (lane & 3);
        double acc = 0.0;
        for (int j = 0; j < L.len[t]; ++j) acc += L.val[128 * t + j] * halo[hp + L.off[128 * t + j]];
        const int32_t i = L.order[L.tile_base[tile] + 64 * t + lane];
        double ref = 0.0, mag = 0.0;
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          ref += A.v[k] * xc[A.ci[k]];
          mag += std::fabs(A.v[k] * xc[A.ci[k]]);
        }
        worst = std::max(worst, std::fabs(acc - ref) / std::max(mag, 1e-300));
        if (A.rp[i + 1] - A.rp[i] != L.len[t]) return fail("stencil row length differs from its class table");
      }
  }
  std::printf("emulated stencil rows: worst relative error %.3e\n", worst);
  if (!(worst < 1e-13)) return fail("emulated stencil differs from A x");
  std::printf("ok\n");
  return 0;
}
