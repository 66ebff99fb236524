// Geometry core of the native grid builder: convex polygons and polyhedra,
// half-space splitting, triangle/box overlap and ray-cast winding numbers.
#pragma once

#include <array>
#include <cmath>
#include <cstdint>
#include <vector>

namespace fvem::geo {

struct V3 {
  double x = 0, y = 0, z = 0;
  V3() = default;
  V3(double a, double b, double c) : x(a), y(b), z(c) {}
  double operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
  double &operator[](int i) { return i == 0 ? x : (i == 1 ? y : z); }
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline V3 operator-(V3 a) { return {-a.x, -a.y, -a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline bool lex_less(V3 a, V3 b) {
  if (a.x != b.x) return a.x < b.x;
  if (a.y != b.y) return a.y < b.y;
  return a.z < b.z;
}

using Polygon = std::vector<V3>;

struct Facet {       // planar convex facet, counter-clockwise about the outward normal
  Polygon p;
  V3 n;              // outward unit normal
  double d = 0;      // n . x = d on the facet
};
using Polyhedron = std::vector<Facet>;

V3 area_vector(const Polygon &P);   // (1/2) sum (p_i - p_0) x (p_{i+1} - p_0)
double area(const Polygon &P);
// part of P with n.x <= d (+tol)
Polygon clip(const Polygon &P, V3 n, double d, double tol = 1e-12);
// part of P inside the convex polyhedron
Polygon clip_to(const Polygon &P, const Polyhedron &C);
// overlap of coplanar convex polygons, Q counter-clockwise about m
Polygon overlap(const Polygon &P, const Polygon &Q, V3 m);
Polyhedron box(V3 lo, V3 hi);
void volume_centroid(const Polyhedron &C, double *vol, V3 *cen);
// split by n.x = d; returns false when the plane does not cut
bool split(const Polyhedron &C, V3 n, double d, Polyhedron *below, Polyhedron *above, double tol = 1e-12);
bool tri_box_overlap(V3 a, V3 b, V3 c, V3 lo, V3 hi);

// Winding number of a closed outward triangle mesh along a slightly tilted +z ray.
class Winding {
 public:
  Winding(const std::vector<V3> &V, const std::vector<std::array<int32_t, 3>> &F, int N);
  int at(V3 p) const;
 private:
  int N_;
  std::vector<V3> a_, e1_, e2_, nrm_;
  std::vector<int64_t> col_ptr_;
  std::vector<int32_t> col_tri_;
};

}  // namespace fvem::geo
