// Virtual-element operators of the native builder (see vem.hpp).
//
// Integration: volume moments of basis monomials by the divergence theorem
// for homogeneous polynomials (int_E f = 1/(3+q) sum_F (n_F.(x_F - x_c)) int_F f
// for f homogeneous of degree q about x_c), face integrals by Radon's
// 7-point degree-5 rule on a fan of triangles (exact for every integrand
// used here, whose degree is at most 3 on faces).
#include "vem.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace fvem::vem {

using geo::cross;
using geo::dot;
using geo::norm;

static const int EXP3[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                                {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
static const int EXP2[6][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2}};

int npoly3(int k) { return k == 1 ? 4 : 10; }
int npoly2(int k) { return k == 1 ? 3 : 6; }

static double ipow(double x, int e) { return e == 0 ? 1.0 : (e == 1 ? x : (e == 2 ? x * x : x * x * x)); }

void Basis::local(V3 x, double y[3]) const {
  const V3 u = x - xc;
  for (int c = 0; c < 3; ++c) y[c] = (u.x * R[0][c] + u.y * R[1][c] + u.z * R[2][c]) / s[c];
}

void Basis::eval(V3 x, int k, double *m) const {
  double y[3];
  local(x, y);
  for (int a = 0; a < npoly3(k); ++a) m[a] = ipow(y[0], EXP3[a][0]) * ipow(y[1], EXP3[a][1]) * ipow(y[2], EXP3[a][2]);
}

void FaceProj::eval(V3 x, int k, double *m) const {
  const V3 u = x - xf;
  const double a = dot(u, t1) / s1, b = dot(u, t2) / s2;
  for (int i = 0; i < npoly2(k); ++i) m[i] = ipow(a, EXP2[i][0]) * ipow(b, EXP2[i][1]);
}

// ------------------------------------------------------------------ small dense helpers

// solve A X = B (A n x n, B n x m, row-major), partial pivoting; B overwritten
static void solve(std::vector<double> A, int n, std::vector<double> &B, int m) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) throw std::runtime_error("singular local projection system");
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
      for (int j = 0; j < m; ++j) std::swap(B[c * m + j], B[piv * m + j]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      for (int j = 0; j < m; ++j) B[r * m + j] -= f * B[c * m + j];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int j = 0; j < m; ++j) {
      double v = B[c * m + j];
      for (int t = c + 1; t < n; ++t) v -= A[c * n + t] * B[t * m + j];
      B[c * m + j] = v / A[c * n + c];
    }
  }
}

// symmetric 3x3 eigenvectors (cyclic Jacobi); returns eigenvalues in w, vectors in columns of V
static void eig3(double A[3][3], double w[3], double V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (std::fabs(A[p][q]) < 1e-300) continue;
        const double th = (A[q][q] - A[p][p]) / (2 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

// ------------------------------------------------------------------ face quadrature (Radon, degree 5)

struct QP {
  V3 x;
  double w;
};

static void polygon_rule(const std::vector<V3> &P, std::vector<QP> &out) {
  static const double s15 = std::sqrt(15.0);
  static const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
  static const double w0 = 9.0 / 40.0, w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  out.clear();
  V3 c;
  for (const V3 &p : P) c = c + p;
  c = (1.0 / static_cast<double>(P.size())) * c;
  const size_t m = P.size();
  for (size_t i = 0; i < m; ++i) {
    const V3 A = c, B = P[i], C = P[(i + 1) % m];
    const double ar = 0.5 * norm(cross(B - A, C - A));
    if (ar == 0) continue;
    auto pt = [&](double l0, double l1, double l2) { return l0 * A + l1 * B + l2 * C; };
    out.push_back({pt(1.0 / 3, 1.0 / 3, 1.0 / 3), w0 * ar});
    const double b1 = 1 - 2 * a1, b2 = 1 - 2 * a2;
    out.push_back({pt(a1, a1, b1), w1 * ar});
    out.push_back({pt(a1, b1, a1), w1 * ar});
    out.push_back({pt(b1, a1, a1), w1 * ar});
    out.push_back({pt(a2, a2, b2), w2 * ar});
    out.push_back({pt(a2, b2, a2), w2 * ar});
    out.push_back({pt(b2, a2, a2), w2 * ar});
  }
}

// ------------------------------------------------------------------ basis choice

static Basis make_basis(const std::vector<V3> &X, V3 xc) {
  Basis b;
  b.xc = xc;
  double hE = 0;
  for (size_t i = 0; i < X.size(); ++i)
    for (size_t j = i + 1; j < X.size(); ++j) hE = std::max(hE, norm(X[i] - X[j]));
  b.hE = hE;
  double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (const V3 &p : X) {
    const V3 u = p - xc;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) C[i][j] += u[i] * u[j];
  }
  double w[3], V[3][3];
  eig3(C, w, V);
  const double wmax = std::max({w[0], w[1], w[2]}), wmin = std::min({w[0], w[1], w[2]});
  // thin when the principal extents differ by more than a factor 4 (variance 16)
  if (wmin <= 0 || wmax > 16.0 * wmin) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) b.R[i][j] = V[i][j];
    for (int c = 0; c < 3; ++c) {
      double e = 0;
      for (const V3 &p : X) e = std::max(e, std::fabs(dot(p - xc, V3(V[0][c], V[1][c], V[2][c]))));
      b.s[c] = e > 0 ? e : hE;
    }
  } else {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) b.R[i][j] = i == j ? 1.0 : 0.0;
    b.s[0] = b.s[1] = b.s[2] = hE;
  }
  return b;
}

// moments int_E y^(a,b,c) for a+b+c <= 2 of a polyhedron given by outward faces
struct Moments {
  double m[3][3][3];
  double at(int a, int b, int c) const { return m[a][b][c]; }
};

static Moments moments(const std::vector<std::vector<V3>> &faces, const Basis &B) {
  Moments M;
  for (auto &a : M.m)
    for (auto &b : a)
      for (double &c : b) c = 0;
  std::vector<QP> q;
  for (const auto &P : faces) {
    const V3 av = geo::area_vector(P);
    const double an = norm(av);
    if (an == 0) continue;
    const V3 n = (1.0 / an) * av;
    const double hf = dot(n, P[0] - B.xc);
    polygon_rule(P, q);
    for (const QP &p : q) {
      double y[3];
      B.local(p.x, y);
      for (int a = 0; a <= 2; ++a)
        for (int b = 0; a + b <= 2; ++b)
          for (int c = 0; a + b + c <= 2; ++c)
            M.m[a][b][c] += hf * p.w * ipow(y[0], a) * ipow(y[1], b) * ipow(y[2], c) / (3.0 + a + b + c);
    }
  }
  return M;
}

// ------------------------------------------------------------------ face projector

FaceProj face_projector(const std::vector<V3> &P, V3 n, int k) {
  FaceProj F;
  const int m = static_cast<int>(P.size());
  F.n = n;
  // area centroid
  double A = 0;
  V3 c;
  for (int i = 1; i + 1 < m; ++i) {
    const double t = 0.5 * dot(cross(P[i] - P[0], P[i + 1] - P[0]), n);
    A += t;
    c = c + t * (P[0] + P[i] + P[i + 1]);
  }
  F.area = A;
  F.xf = (1.0 / (3.0 * A)) * c;
  double hf = 0;
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) hf = std::max(hf, norm(P[i] - P[j]));
  // in-plane frame: principal axes for elongated faces, else first edge
  V3 e0 = P[1] - P[0];
  e0 = (1.0 / norm(e0)) * e0;
  V3 e1 = cross(n, e0);
  double cxx = 0, cxy = 0, cyy = 0;
  for (const V3 &p : P) {
    const double a = dot(p - F.xf, e0), b = dot(p - F.xf, e1);
    cxx += a * a;
    cxy += a * b;
    cyy += b * b;
  }
  const double tr = cxx + cyy, det = cxx * cyy - cxy * cxy;
  const double disc = std::sqrt(std::max(0.0, 0.25 * tr * tr - det));
  const double l1 = 0.5 * tr + disc, l2 = 0.5 * tr - disc;
  if (l2 <= 0 || l1 > 16.0 * l2) {
    double vx = cxy, vy = l1 - cxx;
    if (std::fabs(vx) + std::fabs(vy) < 1e-300) {
      vx = 1;
      vy = 0;
    }
    V3 a1 = vx * e0 + vy * e1;
    a1 = (1.0 / norm(a1)) * a1;
    F.t1 = a1;
    F.t2 = cross(n, a1);
    double s1 = 0, s2 = 0;
    for (const V3 &p : P) {
      s1 = std::max(s1, std::fabs(dot(p - F.xf, F.t1)));
      s2 = std::max(s2, std::fabs(dot(p - F.xf, F.t2)));
    }
    F.s1 = s1 > 0 ? s1 : hf;
    F.s2 = s2 > 0 ? s2 : hf;
  } else {
    F.t1 = e0;
    F.t2 = e1;
    F.s1 = F.s2 = hf;
  }
  const int Nf = npoly2(k);
  const int nd = k == 1 ? m : 2 * m + 1;
  F.nd = nd;
  std::vector<double> D(nd * Nf), B(Nf * nd, 0.0);
  double mv[6];
  for (int i = 0; i < m; ++i) {
    F.eval(P[i], k, mv);
    for (int b = 0; b < Nf; ++b) D[i * Nf + b] = mv[b];
  }
  std::vector<QP> q;
  if (k == 2) {
    for (int i = 0; i < m; ++i) {
      F.eval(0.5 * (P[i] + P[(i + 1) % m]), k, mv);
      for (int b = 0; b < Nf; ++b) D[(m + i) * Nf + b] = mv[b];
    }
    polygon_rule(P, q);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (const QP &p : q) {
      F.eval(p.x, k, mv);
      for (int b = 0; b < Nf; ++b) acc[b] += p.w * mv[b];
    }
    for (int b = 0; b < Nf; ++b) D[2 * m * Nf + b] = acc[b] / A;
    B[0 * nd + 2 * m] = 1.0;
    for (int b = 0; b < Nf; ++b) {
      const double lap = EXP2[b][0] * (EXP2[b][0] - 1) / (F.s1 * F.s1) + EXP2[b][1] * (EXP2[b][1] - 1) / (F.s2 * F.s2);
      B[b * nd + 2 * m] += -lap * A;
    }
  } else {
    for (int i = 0; i < m; ++i) B[0 * nd + i] = 1.0 / m;
  }
  // edge terms: int_e phi (grad m_b . n_e)
  auto grad_n = [&](V3 x, V3 ne, double *g) {
    const V3 u = x - F.xf;
    const double a = dot(u, F.t1) / F.s1, b = dot(u, F.t2) / F.s2;
    const double dt1 = dot(ne, F.t1) / F.s1, dt2 = dot(ne, F.t2) / F.s2;
    for (int i = 0; i < Nf; ++i) {
      const int p = EXP2[i][0], r = EXP2[i][1];
      const double da = p ? p * ipow(a, p - 1) * ipow(b, r) : 0.0;
      const double db = r ? r * ipow(a, p) * ipow(b, r - 1) : 0.0;
      g[i] = da * dt1 + db * dt2;
    }
  };
  for (int i = 0; i < m; ++i) {
    const int j = (i + 1) % m;
    const V3 ev = P[j] - P[i];
    const double L = norm(ev);
    const V3 ne = (1.0 / L) * cross(ev, n);
    double ga[6], gb[6], gm[6];
    grad_n(P[i], ne, ga);
    grad_n(P[j], ne, gb);
    if (k == 1) {
      for (int b = 1; b < Nf; ++b) {
        B[b * nd + i] += 0.5 * L * ga[b];
        B[b * nd + j] += 0.5 * L * gb[b];
      }
    } else {
      grad_n(0.5 * (P[i] + P[j]), ne, gm);
      for (int b = 1; b < Nf; ++b) {
        B[b * nd + i] += L / 6.0 * ga[b];
        B[b * nd + m + i] += 4.0 * L / 6.0 * gm[b];
        B[b * nd + j] += L / 6.0 * gb[b];
      }
    }
  }
  std::vector<double> G(Nf * Nf, 0.0);
  for (int a = 0; a < Nf; ++a)
    for (int b = 0; b < Nf; ++b)
      for (int r = 0; r < nd; ++r) G[a * Nf + b] += B[a * nd + r] * D[r * Nf + b];
  F.Pi = B;
  solve(G, Nf, F.Pi, nd);
  return F;
}

// ------------------------------------------------------------------ cell operators

static void cell_geometry(const Cell &c, std::vector<std::vector<V3>> &fpts, double *vol, V3 *cen) {
  geo::Polyhedron poly;
  fpts.clear();
  for (const auto &cyc : c.faces) {
    std::vector<V3> P;
    for (int v : cyc) P.push_back(c.X[v]);
    fpts.push_back(P);
    geo::Facet f;
    f.p = P;
    poly.push_back(f);
  }
  geo::volume_centroid(poly, vol, cen);
}

static CellData build(const Cell &c, int k, bool stiffness, bool with_div) {
  CellData out;
  out.k = k;
  std::vector<std::vector<V3>> fpts;
  V3 xc;
  cell_geometry(c, fpts, &out.volume, &xc);
  out.basis = make_basis(c.X, xc);
  const Basis &bs = out.basis;
  const Moments M = moments(fpts, bs);
  const int nv = static_cast<int>(c.X.size()), ne = static_cast<int>(c.edges.size());
  const int nf = static_cast<int>(c.faces.size());
  const int nE = c.n_local(k), Nk = npoly3(k);
  // D
  std::vector<double> D(nE * Nk, 0.0);
  double mv[10];
  for (int v = 0; v < nv; ++v) {
    bs.eval(c.X[v], k, mv);
    for (int a = 0; a < Nk; ++a) D[v * Nk + a] = mv[a];
  }
  std::vector<QP> q;
  if (k == 2) {
    for (int e = 0; e < ne; ++e) {
      bs.eval(0.5 * (c.X[c.edges[e][0]] + c.X[c.edges[e][1]]), k, mv);
      for (int a = 0; a < Nk; ++a) D[(nv + e) * Nk + a] = mv[a];
    }
    for (int f = 0; f < nf; ++f) {
      polygon_rule(fpts[f], q);
      double acc[10] = {0}, ar = 0;
      for (const QP &p : q) {
        bs.eval(p.x, k, mv);
        for (int a = 0; a < Nk; ++a) acc[a] += p.w * mv[a];
        ar += p.w;
      }
      for (int a = 0; a < Nk; ++a) D[(nv + ne + f) * Nk + a] = acc[a] / ar;
    }
    for (int a = 0; a < Nk; ++a) D[(nE - 1) * Nk + a] = M.at(EXP3[a][0], EXP3[a][1], EXP3[a][2]) / out.volume;
  }
  // B (right-hand side of the projection)
  std::vector<double> B(Nk * nE, 0.0);
  if (k == 1) {
    for (int v = 0; v < nv; ++v) B[v] = 1.0 / nv;
  } else {
    B[nE - 1] = 1.0;
    for (int a = 1; a < Nk; ++a) {
      double lap = 0;
      for (int d = 0; d < 3; ++d) lap += EXP3[a][d] * (EXP3[a][d] - 1) / (bs.s[d] * bs.s[d]);
      B[a * nE + nE - 1] += -lap * out.volume;
    }
  }
  for (int f = 0; f < nf; ++f) {
    const auto &P = fpts[f];
    const V3 av = geo::area_vector(P);
    const V3 n = (1.0 / norm(av)) * av;
    const FaceProj F = face_projector(P, n, k);
    const int Nf = npoly2(k), nd = F.nd, m = static_cast<int>(P.size());
    // I[b][a] = int_F m^F_b (grad m_a . n)
    std::vector<double> I(Nf * Nk, 0.0);
    polygon_rule(P, q);
    // grad of basis monomials dotted with n: d/dx = sum_d R[:,d]/s_d d/dy_d
    double nd_y[3];
    for (int d = 0; d < 3; ++d) nd_y[d] = (n.x * bs.R[0][d] + n.y * bs.R[1][d] + n.z * bs.R[2][d]) / bs.s[d];
    double mf[6];
    for (const QP &p : q) {
      double y[3];
      bs.local(p.x, y);
      F.eval(p.x, k, mf);
      for (int a = 1; a < Nk; ++a) {
        double g = 0;
        for (int d = 0; d < 3; ++d) {
          const int e = EXP3[a][d];
          if (!e) continue;
          int ex[3] = {EXP3[a][0], EXP3[a][1], EXP3[a][2]};
          ex[d] -= 1;
          g += nd_y[d] * e * ipow(y[0], ex[0]) * ipow(y[1], ex[1]) * ipow(y[2], ex[2]);
        }
        for (int b = 0; b < Nf; ++b) I[b * Nk + a] += p.w * mf[b] * g;
      }
    }
    // face-local DOF -> cell-local DOF
    std::vector<int> loc(nd);
    for (int i = 0; i < m; ++i) loc[i] = c.faces[f][i];
    if (k == 2) {
      for (int i = 0; i < m; ++i) loc[m + i] = nv + c.face_edges[f][i];
      loc[2 * m] = nv + ne + f;
    }
    for (int a = 1; a < Nk; ++a)
      for (int r = 0; r < nd; ++r) {
        double s = 0;
        for (int b = 0; b < Nf; ++b) s += F.Pi[b * nd + r] * I[b * Nk + a];
        B[a * nE + loc[r]] += s;
      }
  }
  // Pi* = (B D)^-1 B
  std::vector<double> G(Nk * Nk, 0.0);
  for (int a = 0; a < Nk; ++a)
    for (int b = 0; b < Nk; ++b)
      for (int r = 0; r < nE; ++r) G[a * Nk + b] += B[a * nE + r] * D[r * Nk + b];
  out.Pis = B;
  solve(G, Nk, out.Pis, nE);
  if (!stiffness) return out;
  // consistency: a(m_a, m_b) from moments; grad m . grad m = sum_d s_d^-2 dy_d m_a dy_d m_b
  std::vector<double> Gt(Nk * Nk, 0.0);
  for (int a = 1; a < Nk; ++a)
    for (int b = 1; b < Nk; ++b) {
      double s = 0;
      for (int d = 0; d < 3; ++d) {
        const int ea = EXP3[a][d], eb = EXP3[b][d];
        if (!ea || !eb) continue;
        int ex[3];
        for (int t = 0; t < 3; ++t) ex[t] = EXP3[a][t] + EXP3[b][t];
        ex[d] -= 2;
        s += ea * eb * M.at(ex[0], ex[1], ex[2]) / (bs.s[d] * bs.s[d]);
      }
      Gt[a * Nk + b] = s;
    }
  out.K.assign(nE * nE, 0.0);
  std::vector<double> T(Nk * nE, 0.0);   // Gt Pi*
  for (int a = 0; a < Nk; ++a)
    for (int r = 0; r < nE; ++r) {
      double s = 0;
      for (int b = 0; b < Nk; ++b) s += Gt[a * Nk + b] * out.Pis[b * nE + r];
      T[a * nE + r] = s;
    }
  for (int r = 0; r < nE; ++r)
    for (int t = 0; t < nE; ++t) {
      double s = 0;
      for (int a = 0; a < Nk; ++a) s += out.Pis[a * nE + r] * T[a * nE + t];
      out.K[r * nE + t] = s;
    }
  // stabilisation h_E (I - Pi)^T (I - Pi), Pi = D Pi*
  std::vector<double> IP(nE * nE);
  for (int r = 0; r < nE; ++r)
    for (int t = 0; t < nE; ++t) {
      double s = 0;
      for (int a = 0; a < Nk; ++a) s += D[r * Nk + a] * out.Pis[a * nE + t];
      IP[r * nE + t] = (r == t ? 1.0 : 0.0) - s;
    }
  for (int r = 0; r < nE; ++r)
    for (int t = 0; t < nE; ++t) {
      double s = 0;
      for (int u = 0; u < nE; ++u) s += IP[u * nE + r] * IP[u * nE + t];
      out.K[r * nE + t] += bs.hE * s;
    }
  if (!with_div) return out;
  // divergence block: b_r = int_E Pi_1 u . grad Pi_k phi_r
  CellData lin = k == 1 ? out : build(c, 1, false, false);
  // same basis frame for both orders
  const std::vector<double> &P1 = lin.Pis;   // 4 x nv
  out.B.assign(nE * 3 * nv, 0.0);
  for (int comp = 0; comp < 3; ++comp) {
    // Mc[a][b] = int_E m1_a d/dx_comp m_b
    double Mc[4][10];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < Nk; ++b) {
        double s = 0;
        for (int d = 0; d < 3; ++d) {
          const int eb = EXP3[b][d];
          if (!eb) continue;
          int ex[3];
          for (int t = 0; t < 3; ++t) ex[t] = EXP3[a][t] + EXP3[b][t];
          ex[d] -= 1;
          s += bs.R[comp][d] / bs.s[d] * eb * M.at(ex[0], ex[1], ex[2]);
        }
        Mc[a][b] = s;
      }
    // B[r][v] = sum_{a,b} Pis[b][r] Mc[a][b] P1[a][v]
    std::vector<double> W(Nk * nv, 0.0);   // W[b][v] = sum_a Mc[a][b] P1[a][v]
    for (int b = 0; b < Nk; ++b)
      for (int v = 0; v < nv; ++v) {
        double s = 0;
        for (int a = 0; a < 4; ++a) s += Mc[a][b] * P1[a * nv + v];
        W[b * nv + v] = s;
      }
    for (int r = 0; r < nE; ++r)
      for (int v = 0; v < nv; ++v) {
        double s = 0;
        for (int b = 0; b < Nk; ++b) s += out.Pis[b * nE + r] * W[b * nv + v];
        out.B[r * (3 * nv) + 3 * v + comp] = s;
      }
  }
  // Velocity correction (Sec. 3.3: Pi_1 u - grad Pi_k p per cell) on the
  // paper's scaled linear monomials z = (x - x_E)/h_E.  Tz maps coefficients
  // on this basis's linear part [1, y] to [1, z]: y_d = sum_i R_id h_E z_i / s_d.
  double Tz[4][4] = {{1, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) Tz[1 + i][1 + d] = bs.R[i][d] * bs.hE / bs.s[d];
  out.V.assign(4 * nv + 12 * nE + 16, 0.0);
  for (int a = 0; a < 4; ++a)
    for (int v = 0; v < nv; ++v) {
      double s = 0;
      for (int b = 0; b < 4; ++b) s += Tz[a][b] * P1[b * nv + v];
      out.V[a * nv + v] = s;
    }
  auto lin_index = [](const int e[3]) {
    for (int a = 0; a < 4; ++a)
      if (EXP3[a][0] == e[0] && EXP3[a][1] == e[1] && EXP3[a][2] == e[2]) return a;
    return -1;
  };
  for (int comp = 0; comp < 3; ++comp) {
    // C[a][b]: d/dx_comp of basis monomial b on the linear monomials [1, y]
    double C[4][10] = {};
    for (int b = 1; b < Nk; ++b)
      for (int d = 0; d < 3; ++d) {
        const int eb = EXP3[b][d];
        if (!eb) continue;
        int ex[3] = {EXP3[b][0], EXP3[b][1], EXP3[b][2]};
        ex[d] -= 1;
        C[lin_index(ex)][b] += bs.R[comp][d] / bs.s[d] * eb;
      }
    // grad_comp Pi_k = T C Pi*
    double TC[4][10] = {};
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < Nk; ++b)
        for (int t = 0; t < 4; ++t) TC[a][b] += Tz[a][t] * C[t][b];
    for (int a = 0; a < 4; ++a)
      for (int r = 0; r < nE; ++r) {
        double s = 0;
        for (int b = 0; b < Nk; ++b) s += TC[a][b] * out.Pis[b * nE + r];
        out.V[4 * nv + (comp * 4 + a) * nE + r] = s;
      }
  }
  // mass of [1, z]: z_i = sum_d R_id s_d y_d / h_E
  double A[4][4] = {};   // A[i][d]: z_i on [1, y]
  A[0][0] = 1.0;
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) A[1 + i][1 + d] = bs.R[i][d] * bs.s[d] / bs.hE;
  double My[4][4];       // int_E of products of [1, y]
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      My[a][b] = M.at(EXP3[a][0] + EXP3[b][0], EXP3[a][1] + EXP3[b][1], EXP3[a][2] + EXP3[b][2]);
  double *Mz = out.V.data() + 4 * nv + 12 * nE;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      double s = 0;
      for (int c2 = 0; c2 < 4; ++c2)
        for (int d = 0; d < 4; ++d) s += A[a][c2] * My[c2][d] * A[b][d];
      Mz[a * 4 + b] = s;
    }
  return out;
}

CellData element(const Cell &c, int k, bool with_div) { return build(c, k, true, with_div); }
CellData projector(const Cell &c, int k) { return build(c, k, false, false); }

void polygon_mean(const std::vector<V3> &P, const Basis &b, int k, double *out) {
  std::vector<QP> q;
  polygon_rule(P, q);
  const int Nk = npoly3(k);
  double mv[10], ar = 0;
  for (int a = 0; a < Nk; ++a) out[a] = 0;
  for (const QP &p : q) {
    b.eval(p.x, k, mv);
    for (int a = 0; a < Nk; ++a) out[a] += p.w * mv[a];
    ar += p.w;
  }
  for (int a = 0; a < Nk; ++a) out[a] /= ar;
}

void polygon_mean_face(const std::vector<V3> &P, const FaceProj &f, int k, double *out) {
  std::vector<QP> q;
  polygon_rule(P, q);
  const int Nf = npoly2(k);
  double mv[6], ar = 0;
  for (int a = 0; a < Nf; ++a) out[a] = 0;
  for (const QP &p : q) {
    f.eval(p.x, k, mv);
    for (int a = 0; a < Nf; ++a) out[a] += p.w * mv[a];
    ar += p.w;
  }
  for (int a = 0; a < Nf; ++a) out[a] /= ar;
}

void polyhedron_mean(const std::vector<std::vector<V3>> &faces, const Basis &b, int k, double *out) {
  const Moments M = moments(faces, b);
  const double vol = M.at(0, 0, 0);
  for (int a = 0; a < npoly3(k); ++a) out[a] = M.at(EXP3[a][0], EXP3[a][1], EXP3[a][2]) / vol;
}

}  // namespace fvem::vem
