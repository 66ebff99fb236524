// Virtual-element operators of orders 1 and 2 on convex polyhedra (native builder).
//
// Paper Sec. 3.1: the projection Pi (orthogonality conditions plus the P0
// constraint: vertex mean for k = 1, cell mean for k = 2), the element
// stiffness consistency + DOF stabilisation; App. A: scaled monomials.
// Sec. 3.2: the projected divergence right-hand side.  Face integrals of
// virtual functions use the face space's own 2-D projection (the 2-D VEM
// obtained by dimensional reduction, Sec. 4).
#pragma once

#include <array>
#include <vector>

#include "geom.hpp"

namespace fvem::vem {

using geo::V3;

// Monomial basis of P_k in y = R^T (x - xc) / s (the paper's basis is R = I,
// s = h_E; thin cells use their principal axes and half-extents, which leaves
// the projection unchanged and keeps the local systems well conditioned).
struct Basis {
  V3 xc;
  double R[3][3];   // columns are the axes
  double s[3];
  double hE;
  void local(V3 x, double y[3]) const;
  void eval(V3 x, int k, double *m) const;   // m[N_k]
};

// A cell with local topology: vertices, edges and outward faces.
struct Cell {
  std::vector<V3> X;                       // local vertices
  std::vector<std::array<int, 2>> edges;   // local vertex pairs
  std::vector<std::vector<int>> faces;     // vertex cycles, counter-clockwise seen from outside
  std::vector<std::vector<int>> face_edges;  // local edge of (cyc[i], cyc[i+1])
  int n_local(int k) const {
    return k == 1 ? static_cast<int>(X.size())
                  : static_cast<int>(X.size() + edges.size() + faces.size() + 1);
  }
};

struct FaceProj {
  V3 xf, t1, t2, n;
  double s1, s2, area;
  std::vector<double> Pi;   // N_f x n_fdof, row-major
  int nd;
  void eval(V3 x, int k, double *m) const;   // face monomials
};

struct CellData {
  int k = 1;
  double volume = 0;
  Basis basis;
  std::vector<double> Pis;   // N_k x n_E
  std::vector<double> K;     // n_E x n_E
  std::vector<double> B;     // n_E x (3 n_v)  (only when requested)
  // velocity-correction block (with B), on the paper's linear monomials
  // z = [1, (x - x_E)/h_E]: Pi_1 (4 x n_v) | grad Pi_k (3 x 4 x n_E) | mass (4 x 4)
  std::vector<double> V;
};

int npoly3(int k);
int npoly2(int k);

// face projector of a planar polygon (counter-clockwise about n)
FaceProj face_projector(const std::vector<V3> &P, V3 n, int k);
// full element data; with_div also builds the divergence block
CellData element(const Cell &c, int k, bool with_div);
// projector only (used for prolongation)
CellData projector(const Cell &c, int k);
// (1/|F|) int_F m over a polygon, in a cell basis
void polygon_mean(const std::vector<V3> &P, const Basis &b, int k, double *out);
void polygon_mean_face(const std::vector<V3> &P, const FaceProj &f, int k, double *out);
// (1/|E|) int_E m over a polyhedron given by outward faces, in a cell basis
void polyhedron_mean(const std::vector<std::vector<V3>> &faces, const Basis &b, int k, double *out);

}  // namespace fvem::vem
