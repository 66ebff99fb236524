"""Velocity correction, loss and chained projections (oracle; test infrastructure).

After the pressure solve the paper corrects the velocity cell by cell: the
projected velocity is Pi_1 u - grad Pi_k p (Sec. 3.3, the G2P update with the
time step folded in, Sec. 3.2).  A cell field is stored as 3 x 4
coefficients per cell on the paper's scaled linear monomials
[1, (x - x_E)/h_E, (y - y_E)/h_E, (z - z_E)/h_E] (App. A), flattened in the
order (cell, velocity component, coefficient).

Readings (the paper defines no loss and has no adjoint):
* loss of a cell field s against a target t: sum_E int_E |s_E - t_E|^2;
* a chained step maps the projected field back to vertex velocities by the
  volume-weighted average of the cells around each vertex, then adds a
  perturbation: u_{k+1}(x_v) = sum_{E ni v} |E| s_{E,k}(x_v) / sum_{E ni v} |E| + eps_k;
  the chain loss is sum_k loss(s_k, t_k) over the projections s_0 .. s_{K-1}.
Gradients are exact reverse mode through the sparse direct solve.
"""
import numpy as np
import scipy.sparse as sp

from .multigrid import direct_solve


def operators(pb):
    """Sparse Pi (12 nc x 3 nv), G (12 nc x n_free), M (12 nc x 12 nc) and Av (3 nv x 12 nc)."""
    cells = pb.asm.cells
    nc, nv, n = len(cells), pb.dofs[0].nv, pb.dofs[0].n_free
    free = pb.dofs[0].free
    pr, pc, pv, gr, gc, gv, mr, mc, mv = [], [], [], [], [], [], [], [], []
    vol = np.zeros(nc)
    X = pb.vertices
    for E, (gd, verts, em, g) in enumerate(cells):
        vol[E] = g.volume
        fd = free[gd]
        keep = fd >= 0
        for c in range(3):
            rows = 12 * E + 4 * c + np.arange(4)
            # Pi_1: coefficients of the linear projection of component c
            pr.append(np.repeat(rows, len(verts)))
            pc.append(np.tile(3 * np.asarray(verts) + c, 4))
            pv.append(em["Pi1s"].ravel())
            # gradient component c of Pi_k p on the linear monomials
            Cc = em["CPis"][c][:, keep]
            gr.append(np.repeat(rows, keep.sum()))
            gc.append(np.tile(fd[keep], 4))
            gv.append(Cc.ravel())
            mr.append(np.repeat(rows, 4))
            mc.append(np.tile(rows, 4))
            mv.append(em["M1"].ravel())
    Pi = sp.csr_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))), shape=(12 * nc, 3 * nv))
    G = sp.csr_matrix((np.concatenate(gv), (np.concatenate(gr), np.concatenate(gc))), shape=(12 * nc, n))
    M = sp.csr_matrix((np.concatenate(mv), (np.concatenate(mr), np.concatenate(mc))), shape=(12 * nc, 12 * nc))
    # vertex averaging: weight |E| / sum of the volumes around the vertex
    W = np.zeros(nv)
    for E, (gd, verts, em, g) in enumerate(cells):
        W[verts] += vol[E]
    ar, ac, av = [], [], []
    for E, (gd, verts, em, g) in enumerate(cells):
        m = np.concatenate([np.ones((len(verts), 1)), (X[verts] - g.xc) / g.hc], axis=1)   # [nv_E, 4]
        w = vol[E] / W[verts]
        for c in range(3):
            ar.append(np.repeat(3 * np.asarray(verts) + c, 4))
            ac.append(np.tile(12 * E + 4 * c + np.arange(4), len(verts)))
            av.append((w[:, None] * m).ravel())
    Av = sp.csr_matrix((np.concatenate(av), (np.concatenate(ar), np.concatenate(ac))), shape=(3 * nv, 12 * nc))
    return {"Pi": Pi, "G": G, "M": M, "Av": Av}


def _ops(pb):
    if not hasattr(pb, "_velocity_ops"):
        pb._velocity_ops = operators(pb)
    return pb._velocity_ops


def project(pb, u):
    """Projected velocity s = Pi_1 u - grad Pi_k p*(u), and the pressure p*."""
    o = _ops(pb)
    p = pb.solve_direct(u)
    return o["Pi"] @ u - o["G"] @ p, p


def loss(pb, s, t):
    o = _ops(pb)
    d = s - t
    return float(d @ (o["M"] @ d))


def project_vjp(pb, gs):
    """g_u = Pi^T g_s + B^T P_perp K^+ P_perp (-G^T g_s): the transpose of u -> s."""
    o = _ops(pb)
    gp = -(o["G"].T @ gs)
    return o["Pi"].T @ gs + pb.adjoint_direct(gp)


def loss_and_gradient(pb, u, t):
    s, _ = project(pb, u)
    o = _ops(pb)
    return loss(pb, s, t), project_vjp(pb, 2.0 * (o["M"] @ (s - t)))


def average(pb, s):
    return _ops(pb)["Av"] @ s


def chain(pb, u0, eps, targets):
    """Loss of K chained projections and its exact gradient with respect to u0."""
    o = _ops(pb)
    u = u0
    ss = []
    total = 0.0
    for k in range(len(targets)):
        s, _ = project(pb, u)
        ss.append(s)
        total += loss(pb, s, targets[k])
        if k + 1 < len(targets):
            u = o["Av"] @ s + eps[k]
    gu_next = None
    for k in reversed(range(len(targets))):
        gs = 2.0 * (o["M"] @ (ss[k] - targets[k]))
        if gu_next is not None:
            gs = gs + o["Av"].T @ gu_next
        gu_next = project_vjp(pb, gs)
    return total, gu_next
