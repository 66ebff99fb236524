"""Exact rational k = 2 VEM projector of an axis-aligned box cell (test helper).

Written directly from the definitions of Sec. 3.1 (local spaces, DOFs,
enhanced face spaces, the projection Pi of the element) in exact rational
arithmetic (SymPy), for cells whose faces are axis-aligned rectangles
(possibly split into sub-faces and carrying hanging vertices).  It shares no
code with the oracle: the projection is basis independent, so the value
functionals it yields can be compared entry by entry with the oracle's
floating-point ones.
"""
import sympy as S

X, Y, Z = S.symbols("x y z")
EXP3 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]


def _rat(p):
    return tuple(S.Rational(c) for c in p)


def _mono3():
    return [X ** a * Y ** b * Z ** c for a, b, c in EXP3]


def _box_integral(f, lo, hi):
    return S.integrate(f, (X, lo[0], hi[0]), (Y, lo[1], hi[1]), (Z, lo[2], hi[2]))


class ExactBoxCell:
    """Local DOFs ordered like the oracle's single-cell geometry: vertices and
    edges in order of first appearance along the face cycles, then faces,
    then the cell mean."""

    def __init__(self, faces, lo, hi):
        self.lo, self.hi = _rat(lo), _rat(hi)
        self.faces = [[_rat(p) for p in cyc] for cyc in faces]
        self.verts = []
        self.edges = []
        for cyc in self.faces:
            for i in range(len(cyc)):
                a, b = cyc[i], cyc[(i + 1) % len(cyc)]
                if a not in self.verts:
                    self.verts.append(a)
                if (a, b) not in self.edges and (b, a) not in self.edges:
                    self.edges.append((a, b))
        self.n = len(self.verts) + len(self.edges) + len(self.faces) + 1
        self.vol = S.Mul(*[h - l for l, h in zip(self.lo, self.hi)])

    # ---- faces: a face is a planar polygon with a constant axis normal
    @staticmethod
    def _face_axes(cyc):
        for ax in range(3):
            if all(p[ax] == cyc[0][ax] for p in cyc):
                return ax
        raise ValueError("face is not axis-aligned")

    def _face_normal(self, cyc):
        ax = self._face_axes(cyc)
        c = cyc[0][ax]
        mid = (self.lo[ax] + self.hi[ax]) / 2
        n = [0, 0, 0]
        n[ax] = 1 if c > mid else -1
        return ax, n

    def face_projector(self, cyc):
        """Pi_f* over the face DOFs (vertices, edge midpoints, face mean) in
        the in-plane monomials (u, v) of the two free coordinates."""
        ax, n = self._face_normal(cyc)
        fr = [a for a in range(3) if a != ax]
        U, V = S.symbols("u v")
        mono = [S.Integer(1), U, V, U ** 2, U * V, V ** 2]
        lo = [min(p[a] for p in cyc) for a in fr]
        hi = [max(p[a] for p in cyc) for a in fr]
        area = (hi[0] - lo[0]) * (hi[1] - lo[1])
        m = len(cyc)
        nd = 2 * m + 1

        def ev(f, p):
            return f.subs({U: p[fr[0]], V: p[fr[1]]})
        D = S.zeros(nd, 6)
        for i, p in enumerate(cyc):
            q = cyc[(i + 1) % m]
            mid = tuple((a + b) / 2 for a, b in zip(p, q))
            for j, f in enumerate(mono):
                D[i, j] = ev(f, p)
                D[m + i, j] = ev(f, mid)
        for j, f in enumerate(mono):
            D[2 * m, j] = S.integrate(f, (U, lo[0], hi[0]), (V, lo[1], hi[1])) / area
        B = S.zeros(6, nd)
        B[0, 2 * m] = 1
        for j, f in enumerate(mono):
            B[j, 2 * m] += -(S.diff(f, U, 2) + S.diff(f, V, 2)) * area
        for i in range(m):
            a, b = cyc[i], cyc[(i + 1) % m]
            d = [b[k] - a[k] for k in range(3)]
            L = S.sqrt(sum(x * x for x in d))
            # outward in-plane edge normal (b - a) x n / |b - a|
            ne = [(d[1] * n[2] - d[2] * n[1]) / L, (d[2] * n[0] - d[0] * n[2]) / L,
                  (d[0] * n[1] - d[1] * n[0]) / L]
            mid = tuple((x + y) / 2 for x, y in zip(a, b))
            for j, f in enumerate(mono):
                g = [S.diff(f, U), S.diff(f, V)]
                gn = lambda p: ev(g[0], p) * ne[fr[0]] + ev(g[1], p) * ne[fr[1]]
                if j == 0:
                    continue
                B[j, i] += L / 6 * gn(a)
                B[j, m + i] += 4 * L / 6 * gn(mid)
                B[j, (i + 1) % m] += L / 6 * gn(b)
        Pis = (B * D).solve(B)
        return Pis, mono, (U, V), fr, n, lo, hi

    def projector(self):
        """Pi* [10 x n] in the monomials x^a y^b z^c (exact rationals)."""
        mono = _mono3()
        nv, ne, nf = len(self.verts), len(self.edges), len(self.faces)
        D = S.zeros(self.n, 10)
        B = S.zeros(10, self.n)
        for i, p in enumerate(self.verts):
            for j, f in enumerate(mono):
                D[i, j] = f.subs({X: p[0], Y: p[1], Z: p[2]})
        for e, (a, b) in enumerate(self.edges):
            mid = tuple((x + y) / 2 for x, y in zip(a, b))
            for j, f in enumerate(mono):
                D[nv + e, j] = f.subs({X: mid[0], Y: mid[1], Z: mid[2]})
        for j, f in enumerate(mono):
            D[self.n - 1, j] = _box_integral(f, self.lo, self.hi) / self.vol
        B[0, self.n - 1] = 1
        for j, f in enumerate(mono):
            B[j, self.n - 1] += -(S.diff(f, X, 2) + S.diff(f, Y, 2) + S.diff(f, Z, 2)) * self.vol
        for fi, cyc in enumerate(self.faces):
            Pif, fm, (U, V), fr, n, flo, fhi = self.face_projector(cyc)
            ax = [a for a in range(3) if a not in fr][0]
            sub = {[X, Y, Z][ax]: cyc[0][ax], [X, Y, Z][fr[0]]: U, [X, Y, Z][fr[1]]: V}
            area = (fhi[0] - flo[0]) * (fhi[1] - flo[1])
            for j, f in enumerate(mono):
                D[nv + ne + fi, j] = S.integrate(f.subs(sub), (U, flo[0], fhi[0]), (V, flo[1], fhi[1])) / area
            m = len(cyc)
            loc = [self.verts.index(p) for p in cyc]
            for i in range(m):
                a, b = cyc[i], cyc[(i + 1) % m]
                e = self.edges.index((a, b)) if (a, b) in self.edges else self.edges.index((b, a))
                loc.append(nv + e)
            loc.append(nv + ne + fi)
            for j, f in enumerate(mono):
                if j == 0:
                    continue
                gn = sum(S.diff(f, s) * n[k] for k, s in enumerate((X, Y, Z))).subs(sub)
                for r, L in enumerate(loc):
                    phi = sum(Pif[b_, r] * fm[b_] for b_ in range(6))
                    B[j, L] += S.integrate(gn * phi, (U, flo[0], fhi[0]), (V, flo[1], fhi[1]))
        G = B * D
        return G.solve(B), mono

    def value_weights(self, Pis, mono, p):
        """Weights of the point value (Pi v)(p) on the local DOFs."""
        p = _rat(p)
        m = S.Matrix([[f.subs({X: p[0], Y: p[1], Z: p[2]}) for f in mono]])
        return m * Pis

    def mean_weights(self, Pis, mono, lo, hi):
        """Weights of the mean of Pi v over the box [lo, hi]."""
        lo, hi = _rat(lo), _rat(hi)
        v = S.Mul(*[b - a for a, b in zip(lo, hi)])
        m = S.Matrix([[_box_integral(f, lo, hi) / v for f in mono]])
        return m * Pis
