"""Turn an oracle problem into the C-ABI problem description (test infrastructure).

The oracle's grid, element matrices and prolongations are handed to the HIP
library unchanged, so the parity tests compare the library's solve with the
oracle's on identical inputs.
"""
import numpy as np


def level_cells(pb, level):
    d = pb.dofs[level]
    ptr = [0]
    dof = []
    for c in range(len(pb.meshes[level].cell_faces)):
        ids = d.free[d.cell_dofs(c)]
        dof.extend(ids.tolist())
        ptr.append(len(dof))
    return np.array(ptr, dtype=np.int64), np.array(dof, dtype=np.int32)


def _canonical_cube_blocks(pb, blocks):
    """Give every uncut cube of one size the same stiffness block.

    The oracle computes each cell's K^E on its own; cubes of equal size then
    differ only by rounding.  Using one computed block for all of them (each
    reordered to the cube's local DOF order by support point) makes
    translated rows of the assembled operator bitwise equal, as the native
    builder's shared blocks do.
    """
    m, d = pb.meshes[0], pb.dofs[0]
    full = _all_points(pb)
    ref = {}
    for c in range(len(m.cell_faces)):
        vts = m.X[m.cell_verts[c]]
        lo, hi = vts.min(axis=0), vts.max(axis=0)
        ext = hi - lo
        if len(m.cell_verts[c]) != 8 or len(m.cell_faces[c]) != 6 or not np.allclose(ext, ext[0], rtol=0, atol=1e-14) \
                or abs(m.cell_volume[c] - ext.prod()) > 1e-14 * ext.prod():
            continue
        key = round(float(ext[0]) * 2 ** 40)
        rel = np.rint((full[d.cell_dofs(c)] - lo) / ext[0] * 4).astype(int)
        keys = [tuple(r) for r in rel]
        if key not in ref:
            ref[key] = (blocks[c], {k: i for i, k in enumerate(keys)})
            continue
        B0, idx = ref[key]
        perm = [idx[k] for k in keys]
        blocks[c] = B0[np.ix_(perm, perm)]
    return blocks


def _all_points(pb, level=0):
    m, d = pb.meshes[level], pb.dofs[level]
    pts = [m.X]
    if d.k == 2:
        pts.append(0.5 * (m.X[m.edges[:, 0]] + m.X[m.edges[:, 1]]))
        pts.append(np.array([m.X[f].mean(axis=0) for f in m.faces]))
        pts.append(np.asarray(m.cell_centroid))
    return np.concatenate(pts)


def describe(pb, canonical_cubes=True):
    L = len(pb.meshes)
    levels = []
    for l in range(L):
        cp, cd = level_cells(pb, l)
        lv = {"n_dof": pb.dofs[l].n_free, "cell_ptr": cp, "cell_dof": cd, "parent": None, "P": None}
        lv["dof_lattice"], lv["lattice_n"] = dof_lattice(pb, l)
        if l + 1 < L:
            lv["parent"] = np.asarray(pb.parents[l], dtype=np.int32)
            P = pb.P[l].tocsr()
            P.sort_indices()
            lv["P"] = (P.indptr.astype(np.int64), P.indices.astype(np.int32), P.data.astype(np.float64))
            lv["P_cols"] = P.shape[1]
        levels.append(lv)
    ke_ptr, ke_val, vptr, vert, be_ptr, be_val = [0], [], [0], [], [0], []
    vc_ptr, vc_val, geom = [0], [], []
    kblocks = [em["K"] for _, _, em, _ in pb.asm.cells]
    if canonical_cubes:
        kblocks = _canonical_cube_blocks(pb, kblocks)
    for (gd, verts, em, g), K in zip(pb.asm.cells, kblocks):
        blk = np.concatenate([em["Pi1s"].ravel(), em["CPis"].ravel(), em["M1"].ravel()])
        vc_val.append(blk)
        vc_ptr.append(vc_ptr[-1] + blk.size)
        geom.append([g.xc[0], g.xc[1], g.xc[2], g.hc, g.volume])
        ke_val.append(K.ravel())
        ke_ptr.append(ke_ptr[-1] + K.size)
        vert.extend(verts.tolist())
        vptr.append(len(vert))
        Bm = em["B"]
        be_val.append(Bm.ravel())
        be_ptr.append(be_ptr[-1] + Bm.size)
    comp = np.full(pb.dofs[0].n_free, -1, dtype=np.int32)
    for c, idx in enumerate(pb.null.floating):
        comp[idx] = c
    return {
        "levels": levels,
        "ke_off": np.array(ke_ptr[:-1], dtype=np.int64), "ke_val": np.concatenate(ke_val),
        "n_vert": pb.dofs[0].nv,
        "cell_vptr": np.array(vptr, dtype=np.int64), "cell_vert": np.array(vert, dtype=np.int32),
        "be_off": np.array(be_ptr[:-1], dtype=np.int64), "be_val": np.concatenate(be_val),
        "component": comp, "n_components": len(pb.null.floating),
        "vc_off": np.array(vc_ptr[:-1], dtype=np.int64), "vc_val": np.concatenate(vc_val),
        "cell_geom": np.array(geom, dtype=np.float64).ravel(),
        "vert_xyz": np.ascontiguousarray(pb.vertices, dtype=np.float64).ravel(),
    }


def dof_points(pb, level=0):
    """Support points of a level's free DOFs: vertices, edge midpoints, face
    vertex means and cell centroids."""
    return _all_points(pb, level)[pb.dofs[level].free_ids]


def dof_lattice(pb, level=0):
    """Integer lattice coordinates of a level's DOFs (-1 off the lattice) on
    the lattice of cells of side 2^level h: the half-lattice of spacing
    2^(level-1) h for k = 2, the vertex lattice for k = 1."""
    span = 2 * pb.w.N if pb.k == 2 else pb.w.N
    if span % 2 ** level or span // 2 ** level < 2:
        return None, 0
    steps = span // 2 ** level
    q = dof_points(pb, level) * steps
    r = np.rint(q)
    on = np.all(np.abs(q - r) < 1e-7, axis=1) & np.all((r >= 0) & (r <= steps), axis=1)
    lat = np.where(on[:, None], r, -1).astype(np.int32)
    return lat.ravel(), int(steps + 1)
