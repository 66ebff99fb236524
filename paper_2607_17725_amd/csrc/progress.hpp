// Setup progress lines on stderr, printed when FVEM_VERBOSE is set to a
// non-empty value other than "0".  Large grids take minutes to build; the
// lines let a caller tell a long setup from a stuck one.
#pragma once

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>

namespace fvem {

inline bool verbose() {
  static const bool v = [] {
    const char *e = std::getenv("FVEM_VERBOSE");
    return e && e[0] && !(e[0] == '0' && e[1] == 0);
  }();
  return v;
}

inline void progress(const char *fmt, ...) {
  if (!verbose()) return;
  static const auto t0 = std::chrono::steady_clock::now();
  const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::fprintf(stderr, "[fvem %7.1fs] ", t);
  va_list ap;
  va_start(ap, fmt);
  std::vfprintf(stderr, fmt, ap);
  va_end(ap);
  std::fputc('\n', stderr);
  std::fflush(stderr);
}

}  // namespace fvem
