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


def describe(pb):
    L = len(pb.meshes)
    levels = []
    for l in range(L):
        cp, cd = level_cells(pb, l)
        lv = {"n_dof": pb.dofs[l].n_free, "cell_ptr": cp, "cell_dof": cd, "parent": None, "P": None}
        if l + 1 < L:
            lv["parent"] = np.asarray(pb.parents[l], dtype=np.int32)
            P = pb.P[l].tocsr()
            P.sort_indices()
            lv["P"] = (P.indptr.astype(np.int64), P.indices.astype(np.int32), P.data.astype(np.float64))
            lv["P_cols"] = P.shape[1]
        levels.append(lv)
    ke_ptr, ke_val, vptr, vert, be_ptr, be_val = [0], [], [0], [], [0], []
    vc_ptr, vc_val, geom = [0], [], []
    for gd, verts, em, g in pb.asm.cells:
        blk = np.concatenate([em["Pi1s"].ravel(), em["CPis"].ravel(), em["M1"].ravel()])
        vc_val.append(blk)
        vc_ptr.append(vc_ptr[-1] + blk.size)
        geom.append([g.xc[0], g.xc[1], g.xc[2], g.hc, g.volume])
        K = em["K"]
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
