// Geometry core of the native grid builder (see geom.hpp).
#include "geom.hpp"

#include <algorithm>

namespace fvem::geo {

V3 area_vector(const Polygon &P) {
  // fan about the first vertex: relative positions keep tiny faces far from
  // the origin exact instead of cancelling to zero
  V3 s;
  const size_t m = P.size();
  for (size_t i = 1; i + 1 < m; ++i) s = s + cross(P[i] - P[0], P[i + 1] - P[0]);
  return 0.5 * s;
}

double area(const Polygon &P) { return norm(area_vector(P)); }

static V3 plane_point(V3 a, V3 b, double sa, double sb) {
  if (lex_less(b, a)) {
    std::swap(a, b);
    std::swap(sa, sb);
  }
  const double t = sa / (sa - sb);
  return a + t * (b - a);
}

static Polygon dedupe(Polygon out) {
  Polygon keep;
  for (const V3 &p : out)
    if (keep.empty() || norm(p - keep.back()) > 1e-13) keep.push_back(p);
  while (keep.size() > 1 && norm(keep.front() - keep.back()) <= 1e-13) keep.pop_back();
  if (keep.size() < 3) keep.clear();
  return keep;
}

Polygon clip(const Polygon &P, V3 n, double d, double tol) {
  const size_t m = P.size();
  if (m == 0) return {};
  std::vector<double> s(m);
  for (size_t i = 0; i < m; ++i) s[i] = dot(n, P[i]) - d;
  Polygon out;
  out.reserve(m + 2);
  for (size_t i = 0; i < m; ++i) {
    const size_t j = (i + 1) % m;
    if (s[i] <= tol) out.push_back(P[i]);
    if ((s[i] < -tol && s[j] > tol) || (s[i] > tol && s[j] < -tol)) out.push_back(plane_point(P[i], P[j], s[i], s[j]));
  }
  if (out.size() < 3) return {};
  return dedupe(std::move(out));
}

Polygon clip_to(const Polygon &P, const Polyhedron &C) {
  Polygon Q = P;
  for (const Facet &f : C) {
    Q = clip(Q, f.n, f.d);
    if (Q.size() < 3) return {};
  }
  return Q;
}

Polygon overlap(const Polygon &P, const Polygon &Q, V3 m) {
  Polygon R = P;
  const size_t q = Q.size();
  for (size_t i = 0; i < q; ++i) {
    V3 on = cross(Q[(i + 1) % q] - Q[i], m);
    const double l = norm(on);
    if (l == 0) continue;
    on = (1.0 / l) * on;
    R = clip(R, on, dot(on, Q[i]));
    if (R.size() < 3) return {};
  }
  return R;
}

Polyhedron box(V3 lo, V3 hi) {
  const double x0 = lo.x, y0 = lo.y, z0 = lo.z, x1 = hi.x, y1 = hi.y, z1 = hi.z;
  Polyhedron C(6);
  C[0] = {{{x0, y0, z0}, {x0, y0, z1}, {x0, y1, z1}, {x0, y1, z0}}, {-1, 0, 0}, -x0};
  C[1] = {{{x1, y0, z0}, {x1, y1, z0}, {x1, y1, z1}, {x1, y0, z1}}, {1, 0, 0}, x1};
  C[2] = {{{x0, y0, z0}, {x1, y0, z0}, {x1, y0, z1}, {x0, y0, z1}}, {0, -1, 0}, -y0};
  C[3] = {{{x0, y1, z0}, {x0, y1, z1}, {x1, y1, z1}, {x1, y1, z0}}, {0, 1, 0}, y1};
  C[4] = {{{x0, y0, z0}, {x0, y1, z0}, {x1, y1, z0}, {x1, y0, z0}}, {0, 0, -1}, -z0};
  C[5] = {{{x0, y0, z1}, {x1, y0, z1}, {x1, y1, z1}, {x0, y1, z1}}, {0, 0, 1}, z1};
  return C;
}

void volume_centroid(const Polyhedron &C, double *vol, V3 *cen) {
  V3 o;
  size_t cnt = 0;
  for (const Facet &f : C)
    for (const V3 &p : f.p) {
      o = o + p;
      ++cnt;
    }
  o = (1.0 / static_cast<double>(cnt)) * o;
  double v = 0;
  V3 c;
  for (const Facet &f : C) {
    V3 fc;
    for (const V3 &p : f.p) fc = fc + p;
    fc = (1.0 / static_cast<double>(f.p.size())) * fc;
    const size_t m = f.p.size();
    for (size_t i = 0; i < m; ++i) {
      const V3 a = f.p[i] - o, b = f.p[(i + 1) % m] - o, e = fc - o;
      const double t = dot(e, cross(a, b)) / 6.0;
      v += t;
      c = c + t * (a + b + e);
    }
  }
  *vol = v;
  *cen = v != 0 ? o + (1.0 / (4.0 * v)) * c : o;
}

static Polygon order_ccw(std::vector<V3> pts, V3 n) {
  V3 c;
  for (const V3 &p : pts) c = c + p;
  c = (1.0 / static_cast<double>(pts.size())) * c;
  V3 t1 = pts[0] - c;
  t1 = (1.0 / norm(t1)) * t1;
  const V3 t2 = cross(n, t1);
  std::vector<std::pair<double, size_t>> ang(pts.size());
  for (size_t i = 0; i < pts.size(); ++i) ang[i] = {std::atan2(dot(pts[i] - c, t2), dot(pts[i] - c, t1)), i};
  std::stable_sort(ang.begin(), ang.end(), [](auto &a, auto &b) { return a.first < b.first; });
  Polygon out;
  for (auto &a : ang) out.push_back(pts[a.second]);
  return out;
}

bool split(const Polyhedron &C, V3 n, double d, Polyhedron *below, Polyhedron *above, double tol) {
  double smin = 1e300, smax = -1e300;
  for (const Facet &f : C)
    for (const V3 &p : f.p) {
      const double s = dot(n, p) - d;
      smin = std::min(smin, s);
      smax = std::max(smax, s);
    }
  if (smax <= tol || smin >= -tol) return false;
  below->clear();
  above->clear();
  std::vector<V3> cap;
  for (const Facet &f : C) {
    const size_t m = f.p.size();
    std::vector<double> s(m);
    for (size_t i = 0; i < m; ++i) s[i] = dot(n, f.p[i]) - d;
    for (size_t i = 0; i < m; ++i) {
      const size_t j = (i + 1) % m;
      if (std::fabs(s[i]) <= tol) cap.push_back(f.p[i]);
      if ((s[i] < -tol && s[j] > tol) || (s[i] > tol && s[j] < -tol))
        cap.push_back(plane_point(f.p[i], f.p[j], s[i], s[j]));
    }
    Polygon lo = clip(f.p, n, d, tol), hi = clip(f.p, -n, -d, tol);
    if (lo.size() >= 3 && area(lo) > 0) below->push_back({lo, f.n, f.d});
    if (hi.size() >= 3 && area(hi) > 0) above->push_back({hi, f.n, f.d});
  }
  std::vector<V3> uniq;
  for (const V3 &p : cap) {
    bool dup = false;
    for (const V3 &q : uniq)
      if (norm(p - q) <= 1e-13) {
        dup = true;
        break;
      }
    if (!dup) uniq.push_back(p);
  }
  if (uniq.size() >= 3) {
    below->push_back({order_ccw(uniq, n), n, d});
    above->push_back({order_ccw(uniq, -n), -n, -d});
  }
  return true;
}

bool tri_box_overlap(V3 a, V3 b, V3 c, V3 lo, V3 hi) {
  const V3 ctr = 0.5 * (lo + hi);
  const double eps = 1e-12;
  const V3 half = 0.5 * (hi - lo) + V3(eps, eps, eps);
  const V3 v[3] = {a - ctr, b - ctr, c - ctr};
  const V3 e[3] = {v[1] - v[0], v[2] - v[1], v[0] - v[2]};
  for (int i = 0; i < 3; ++i) {
    const double mn = std::min({v[0][i], v[1][i], v[2][i]}), mx = std::max({v[0][i], v[1][i], v[2][i]});
    if (mn > half[i] || mx < -half[i]) return false;
  }
  const V3 n = cross(e[0], e[1]);
  const double r = half.x * std::fabs(n.x) + half.y * std::fabs(n.y) + half.z * std::fabs(n.z);
  if (std::fabs(dot(n, v[0])) > r) return false;
  const V3 ax[3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3 a2 = cross(ax[i], e[j]);
      if (dot(a2, a2) < 1e-300) continue;
      const double p0 = dot(a2, v[0]), p1 = dot(a2, v[1]), p2 = dot(a2, v[2]);
      const double rr = half.x * std::fabs(a2.x) + half.y * std::fabs(a2.y) + half.z * std::fabs(a2.z);
      if (std::min({p0, p1, p2}) > rr || std::max({p0, p1, p2}) < -rr) return false;
    }
  return true;
}

// tilted ray direction: a generic small tilt avoids grazing shared edges of
// triangles laid out on the background lattice
static const V3 kRay = [] {
  V3 d(3.1e-5 * std::sqrt(2.0), 1.7e-5 * std::sqrt(3.0), 1.0);
  return (1.0 / norm(d)) * d;
}();

Winding::Winding(const std::vector<V3> &V, const std::vector<std::array<int32_t, 3>> &F, int N) : N_(N) {
  const size_t nt = F.size();
  a_.resize(nt);
  e1_.resize(nt);
  e2_.resize(nt);
  nrm_.resize(nt);
  const double h = 1.0 / N, pad = 1e-3 * h + 1e-4;
  std::vector<std::vector<int32_t>> cols(static_cast<size_t>(N) * N);
  for (size_t t = 0; t < nt; ++t) {
    const V3 a = V[F[t][0]], b = V[F[t][1]], c = V[F[t][2]];
    a_[t] = a;
    e1_[t] = b - a;
    e2_[t] = c - a;
    nrm_[t] = cross(e1_[t], e2_[t]);
    const double xl = std::min({a.x, b.x, c.x}) - pad, xh = std::max({a.x, b.x, c.x}) + pad;
    const double yl = std::min({a.y, b.y, c.y}) - pad, yh = std::max({a.y, b.y, c.y}) + pad;
    const int i0 = std::clamp(static_cast<int>(std::floor(xl / h)), 0, N - 1);
    const int i1 = std::clamp(static_cast<int>(std::floor(xh / h)), 0, N - 1);
    const int j0 = std::clamp(static_cast<int>(std::floor(yl / h)), 0, N - 1);
    const int j1 = std::clamp(static_cast<int>(std::floor(yh / h)), 0, N - 1);
    for (int i = i0; i <= i1; ++i)
      for (int j = j0; j <= j1; ++j) cols[static_cast<size_t>(i) * N + j].push_back(static_cast<int32_t>(t));
  }
  col_ptr_.assign(cols.size() + 1, 0);
  for (size_t k = 0; k < cols.size(); ++k) col_ptr_[k + 1] = col_ptr_[k] + static_cast<int64_t>(cols[k].size());
  col_tri_.reserve(col_ptr_.back());
  for (auto &c : cols) col_tri_.insert(col_tri_.end(), c.begin(), c.end());
}

int Winding::at(V3 p) const {
  const double h = 1.0 / N_;
  const int i = std::clamp(static_cast<int>(p.x / h), 0, N_ - 1);
  const int j = std::clamp(static_cast<int>(p.y / h), 0, N_ - 1);
  const size_t k = static_cast<size_t>(i) * N_ + j;
  int w = 0;
  for (int64_t q = col_ptr_[k]; q < col_ptr_[k + 1]; ++q) {
    const int32_t t = col_tri_[q];
    const V3 pv = cross(kRay, e2_[t]);
    const double det = dot(e1_[t], pv);
    if (std::fabs(det) < 1e-300) continue;
    const double inv = 1.0 / det;
    const V3 tv = p - a_[t];
    const double u = dot(tv, pv) * inv;
    if (u < 0 || u > 1) continue;
    const V3 qv = cross(tv, e1_[t]);
    const double v = dot(kRay, qv) * inv;
    if (v < 0 || u + v > 1) continue;
    const double tt = dot(e2_[t], qv) * inv;
    if (tt <= 0) continue;
    w += dot(nrm_[t], kRay) > 0 ? 1 : -1;
  }
  return w;
}

}  // namespace fvem::geo
