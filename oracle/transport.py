"""The steps on either side of the pressure solve in the simulation loop
(Algorithm 1), as a plain FP64 statement (oracle; test infrastructure).

One step of the loop:
1. P2G (Sec. 3.2): each velocity DOF (a vertex of the finest grid) takes the
   normalised radial-kernel average of the values carried by the particles,
   f_i = sum_p f_p w_ip / sum_p w_ip with w_ip = k(|x_p - x_i|^2 / R^2),
   k(q) = max(0, 1 - q)^3 and R the background grid spacing h.
2. Force (Sec. 3.2): u' = u + f dt at the DOF level, f from the Boussinesq
   buoyancy of the transferred smoke density and temperature.
3. The projection: p solves K p = B u' (Delta t folded in), and the projected
   velocity is the per-cell linear polynomial Pi_1 u' - grad Pi_k p (Sec. 3.3).
4. G2P (Sec. 3.3): the polynomial velocity increment Pi_1 u_new - Pi_1 u
   (u: the P2G velocity before the force) updates particle velocities by a
   FLIP/PIC blend.
5. Advection (Sec. 3.3): second-order Runge-Kutta through the grid velocity
   Pi_1 u_new, with mirror reflection of particles that leave the fluid.

Readings (the paper leaves these open, or prints them inconsistently):
* a vertex with no particle inside its kernel support gets the value 0;
* buoyancy f = (-alpha rho + beta T) e_z, with +z up;
* the blend is the standard one the paper cites, u_p <- a (u_p + du(x_p)) +
  (1 - a) u_new(x_p); the printed formula leaves the factor a off du, which
  would count du twice in the PIC limit a = 0;
* particles that start outside the fluid are ghosts: they take part in P2G
  with the values they carry and are never updated or moved (Sec. 6 setup);
* RK2 is the midpoint rule; the step is cut into n = max(1, ceil(dt v / h))
  substeps for a CFL number of 1, v the largest grid speed at the particles;
* a stage that ends outside the fluid is reflected in the plane of the first
  boundary crossing along it (obstacle triangle or box wall), up to four
  times; a point still outside after that stays where the stage began.  A
  uniform grid of triangle lists stands in for the paper's AABB tree.
"""
import math

import numpy as np


# ----------------------------------------------------------------- P2G, force

def kernel(q):
    """k(q) = max(0, 1 - q)^3 (Sec. 3.2)."""
    return np.maximum(0.0, 1.0 - q) ** 3


def p2g(X, xp, fp, R):
    """Values at points X [nv, 3] from particles at xp [np, 3] carrying fp [np, m]."""
    X = np.asarray(X, dtype=np.float64)
    xp = np.asarray(xp, dtype=np.float64)
    fp = np.asarray(fp, dtype=np.float64).reshape(len(xp), -1)
    out = np.zeros((len(X), fp.shape[1]))
    for a in range(0, len(X), 256):
        d2 = ((X[a:a + 256, None, :] - xp[None, :, :]) ** 2).sum(axis=2)
        w = kernel(d2 / (R * R))
        den = w.sum(axis=1)
        num = w @ fp
        ok = den > 0
        out[a:a + 256][ok] = num[ok] / den[ok, None]
    return out


def buoyancy(u, rho, temp, alpha, beta, dt):
    """u' = u + dt f at the vertices, f = (-alpha rho + beta T) e_z."""
    v = np.array(u, dtype=np.float64).reshape(-1, 3)
    v[:, 2] += dt * (-alpha * np.asarray(rho) + beta * np.asarray(temp))
    return v.ravel()


# ------------------------------------------------------------ point location

class Locator:
    """Level-0 cell holding a point: the cells are convex, so a point is in a
    cell when it lies on the inner side of every face plane of the cell."""

    TOL = 1e-12

    def __init__(self, pb):
        m = pb.meshes[0]
        self.N = pb.w.N
        self.cells_of_bg = {}
        self.planes = []
        for c in range(len(m.cell_faces)):
            n_out, off = [], []
            for f, o in m.cell_faces[c]:
                n = o * np.asarray(m.face_normal[f])
                n_out.append(n)
                off.append(float(n @ m.X[m.faces[f][0]]))
            self.planes.append((np.array(n_out), np.array(off)))
            bg = tuple(np.clip(np.floor(m.cell_centroid[c] * self.N).astype(int), 0, self.N - 1))
            self.cells_of_bg.setdefault(bg, []).append(c)

    def cell_of(self, x):
        x = np.asarray(x, dtype=np.float64)
        if np.any(x < 0.0) or np.any(x > 1.0):
            return -1
        bg = tuple(np.clip(np.floor(x * self.N).astype(int), 0, self.N - 1))
        for c in self.cells_of_bg.get(bg, ()):
            n, off = self.planes[c]
            if np.all(n @ x - off <= self.TOL):
                return c
        return -1


# ---------------------------------------------------- grid velocity, G2P

def eval_field(pb, s, c, x):
    """Cell c's linear velocity at x from its 3 x 4 coefficients on
    [1, (x - x_E)/h_E] (App. A scaled monomials)."""
    g = pb.asm.cells[c][3]
    z = np.concatenate([[1.0], (np.asarray(x) - g.xc) / g.hc])
    return np.asarray(s[12 * c:12 * c + 12]).reshape(3, 4) @ z


def g2p(pb, loc, xp, up, s_new, s_old, a_flip, ghost):
    """FLIP/PIC update of the particle velocities (Sec. 3.3, standard blend)."""
    out = np.array(up, dtype=np.float64).reshape(-1, 3)
    for p in range(len(xp)):
        if ghost[p]:
            continue
        c = loc.cell_of(xp[p])
        if c < 0:
            continue
        unew = eval_field(pb, s_new, c, xp[p])
        du = unew - eval_field(pb, s_old, c, xp[p])
        out[p] = a_flip * (out[p] + du) + (1.0 - a_flip) * unew
    return out


# -------------------------------------------------------------- advection

def _first_crossing(a, b, tri):
    """Smallest t in (0, 1] where the segment a -> b meets a triangle of tri
    [nt, 3, 3] or leaves the unit box; returns (t, unit normal) or None."""
    best = None
    d = b - a
    for ax in range(3):
        for wall in (0.0, 1.0):
            if d[ax] != 0.0:
                t = (wall - a[ax]) / d[ax]
                if 1e-12 < t <= 1.0 and (best is None or t < best[0]):
                    n = np.zeros(3)
                    n[ax] = 1.0
                    best = (t, n)
    if len(tri):
        p0, e1, e2 = tri[:, 0], tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]
        pv = np.cross(d, e2)
        det = np.einsum("ij,ij->i", e1, pv)
        ok = np.abs(det) > 1e-300
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        tv = a - p0
        uu = np.einsum("ij,ij->i", tv, pv) * inv
        qv = np.cross(tv, e1)
        vv = (qv @ d) * inv
        tt = np.einsum("ij,ij->i", e2, qv) * inv
        hit = ok & (uu >= 0) & (vv >= 0) & (uu + vv <= 1) & (tt > 1e-12) & (tt <= 1.0)
        if hit.any():
            j = np.nonzero(hit)[0][np.argmin(tt[hit])]
            if best is None or tt[j] < best[0]:
                n = np.cross(e1[j], e2[j])
                best = (float(tt[j]), n / np.linalg.norm(n))
    return best


def resolve(loc, tri, a, b):
    """End point of a stage a -> b after mirror reflection (reading above)."""
    a0 = np.array(a, dtype=np.float64)
    a = a0.copy()
    b = np.array(b, dtype=np.float64)
    for _ in range(4):
        if loc.cell_of(b) >= 0:
            return b
        hit = _first_crossing(a, b, tri)
        if hit is None:
            return a0
        t, n = hit
        q = a + t * (b - a)
        b = b - 2.0 * ((b - q) @ n) * n
        a = q
    return b if loc.cell_of(b) >= 0 else a0


def grid_speed_max(pb, loc, xp, s, ghost):
    v = 0.0
    for p in range(len(xp)):
        if ghost[p]:
            continue
        c = loc.cell_of(xp[p])
        if c >= 0:
            v = max(v, float(np.linalg.norm(eval_field(pb, s, c, xp[p]))))
    return v


def substeps(vmax, dt, h):
    return max(1, int(math.ceil(dt * vmax / h)))


def advect(pb, loc, tri, xp, s, dt, ghost):
    """Midpoint RK2 through the grid velocity s, CFL-1 substeps, reflection."""
    h = 1.0 / pb.w.N
    x = np.array(xp, dtype=np.float64).reshape(-1, 3)
    n = substeps(grid_speed_max(pb, loc, x, s, ghost), dt, h)
    tau = dt / n

    def vel(y):
        c = loc.cell_of(y)
        return eval_field(pb, s, c, y) if c >= 0 else np.zeros(3)

    for _ in range(n):
        for p in range(len(x)):
            if ghost[p]:
                continue
            a = x[p]
            if loc.cell_of(a) < 0:
                continue
            mid = resolve(loc, tri, a, a + 0.5 * tau * vel(a))
            x[p] = resolve(loc, tri, a, a + tau * vel(mid))
    return x, n


# ------------------------------------------------------------ a whole step

def step(pb, loc, xp, up, rho, temp, ghost, dt, a_flip, alpha, beta):
    """One simulation step; returns new positions, velocities and the pieces
    (vertex fields, projected velocities, pressure, substeps)."""
    from .velocity import operators
    V, F = pb.boundary
    tri = np.asarray(V, dtype=np.float64)[np.asarray(F)]
    h = 1.0 / pb.w.N
    f = p2g(pb.vertices, xp, np.column_stack([np.asarray(up).reshape(-1, 3), rho, temp]), h)
    u = f[:, :3].ravel()
    u1 = buoyancy(u, f[:, 3], f[:, 4], alpha, beta, dt)
    ops = operators(pb)
    p = pb.solve_direct(u1)
    s_new = ops["Pi"] @ u1 - ops["G"] @ p
    s_old = ops["Pi"] @ u
    up2 = g2p(pb, loc, xp, up, s_new, s_old, a_flip, ghost)
    xp2, n = advect(pb, loc, tri, xp, s_new, dt, ghost)
    return xp2, up2, {"vertex": f, "u_forced": u1, "p": p, "s_new": s_new, "s_old": s_old, "substeps": n}
