// Host-only run of the native grid builder (cut cells, hierarchy, VEM
// operators, prolongation) on a boundary mesh read from files, for a build
// with the address and undefined-behaviour sanitizers.  Prints the level
// sizes and exits non-zero when an invariant fails: every cell's DOF list
// and parent in range, prolongation columns in range, operators finite.
// Built with g++ by tests/test_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2607_17725_amd/csrc/grid.hpp"

template <typename T>
static std::vector<T> read_file(const char *path) {
  std::FILE *f = std::fopen(path, "rb");
  if (!f) std::exit(2);
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
  if (argc != 6) return fail("usage: V F N k levels");
  const std::vector<double> V = read_file<double>(argv[1]);
  const std::vector<int32_t> F = read_file<int32_t>(argv[2]);
  fvem::grid::Input in;
  in.V = V.data();
  in.nv = static_cast<int64_t>(V.size() / 3);
  in.F = F.data();
  in.nt = static_cast<int64_t>(F.size() / 3);
  in.N = std::atoi(argv[3]);
  in.k = std::atoi(argv[4]);
  in.L = std::atoi(argv[5]);
  fvem::grid::Output out;
  fvem::grid::build_grid(in, &out);
  const size_t L = out.levels.size();
  for (size_t l = 0; l < L; ++l) {
    const auto &lv = out.levels[l];
    std::printf("level %zu: %lld cells, %lld DOFs\n", l, static_cast<long long>(lv.n_cells),
                static_cast<long long>(lv.n_dof));
    for (int32_t d : lv.cell_dof)
      if (d < -1 || d >= lv.n_dof) return fail("cell DOF out of range");
    if (l + 1 < L) {
      for (int32_t p : lv.parent)
        if (p < 0 || p >= out.levels[l + 1].n_cells) return fail("parent out of range");
      const auto &P = out.P[l];
      for (int32_t c : P.ci)
        if (c < 0 || c >= out.levels[l + 1].n_dof) return fail("prolongation column out of range");
      for (double v : P.v)
        if (!std::isfinite(v)) return fail("prolongation value not finite");
    }
  }
  for (double v : out.ke_val)
    if (!std::isfinite(v)) return fail("element stiffness not finite");
  std::printf("ok\n");
  return 0;
}
