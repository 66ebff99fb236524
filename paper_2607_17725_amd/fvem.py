"""ctypes binding of libfvem.so (the C ABI in include/fvem.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory and the stream.  There is no fallback: if the
library is missing or no GPU is visible, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfvem.so")

STATUS = {0: "OK", 1: "INVALID", 2: "HIP", 3: "OOM", 4: "NOT_SPD", 5: "NOT_CONVERGED", 6: "NONFINITE",
          7: "BUSY"}
OP_K, OP_B, OP_BT, OP_VCYCLE, OP_VCYCLE32, OP_PROJECT = range(6)
OP_PI1, OP_PI1T, OP_G, OP_GT, OP_MASS, OP_AV, OP_AVT = range(6, 13)
APPLY_ACCUMULATE = 0x100
GRID_NAIVE_PROLONGATION = 0x1
PREC_FP64, PREC_MIXED = 0, 1
INPUT_VELOCITY, INPUT_RHS = 0, 1


class FvemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fvem {STATUS.get(code, code)}: {msg}")
        self.code = code


class NotConverged(FvemError):
    pass


class _CSR(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Level(ctypes.Structure):
    _fields_ = [("n_dof", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("cell_ptr", ctypes.c_void_p),
                ("cell_dof", ctypes.c_void_p), ("parent", ctypes.c_void_p), ("P", _CSR),
                ("dof_lattice", ctypes.c_void_p), ("lattice_n", ctypes.c_int32)]


class _Grid(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("levels", ctypes.POINTER(_Level)),
                ("ke_off", ctypes.c_void_p), ("ke_val", ctypes.c_void_p), ("ke_len", ctypes.c_int64),
                ("n_vert", ctypes.c_int64), ("cell_vptr", ctypes.c_void_p), ("cell_vert", ctypes.c_void_p),
                ("be_off", ctypes.c_void_p), ("be_val", ctypes.c_void_p), ("be_len", ctypes.c_int64),
                ("component", ctypes.c_void_p), ("n_components", ctypes.c_int32),
                ("vc_off", ctypes.c_void_p), ("vc_val", ctypes.c_void_p), ("vc_len", ctypes.c_int64),
                ("cell_geom", ctypes.c_void_p), ("vert_xyz", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("cheb_degree", ctypes.c_int32), ("cheb_lower", ctypes.c_double),
                ("coarse_dense_max", ctypes.c_int32), ("coarse_rcond", ctypes.c_double),
                ("coarse_shift", ctypes.c_double), ("small_level_rows", ctypes.c_int64),
                ("max_templates", ctypes.c_int32), ("lattice_min_fraction", ctypes.c_double),
                ("column_codes", ctypes.c_int32), ("galerkin_general", ctypes.c_int32),
                ("vcycle_graphs", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("input", ctypes.c_int32), ("replace_every", ctypes.c_int32), ("profile", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_fine_smoother", ctypes.c_double), ("n_fine_smoother", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("ms_vcycle", ctypes.c_double), ("n_vcycle", ctypes.c_int32),
                ("ms_fine_stencil", ctypes.c_double), ("n_fine_stencil", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ["fvem_hierarchy_build", "fvem_solve", "fvem_solve_adjoint", "fvem_apply", "fvem_level_matrix",
           "fvem_hierarchy_info", "fvem_hierarchy_destroy", "fvem_last_error", "fvem_grid_build",
           "fvem_grid_describe", "fvem_grid_info", "fvem_grid_level_points", "fvem_grid_destroy",
           "fvem_project_velocity", "fvem_project_velocity_adjoint", "fvem_velocity_loss", "fvem_hierarchy_cells",
           "fvem_level_storage", "fvem_level_bytes", "fvem_project_noalloc", "fvem_level_stencil",
           "fvem_transfer_storage", "fvem_vcycle_bytes", "fvem_level_slices",
           "fvem_memory_breakdown", "fvem_grid_build_ex", "fvem_transport_create", "fvem_transport_destroy",
           "fvem_locate", "fvem_p2g", "fvem_buoyancy", "fvem_g2p", "fvem_advect", "fvem_grid_cell_faces"]

_lib = None


def load(path=LIB_PATH):
    """Load libfvem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FvemError(1, f"{path} is missing: build it with paper_2607_17725_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.fvem_hierarchy_build.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Options), vp, ctypes.POINTER(vp)]
    lib.fvem_hierarchy_build.restype = ctypes.c_int
    for fn in (lib.fvem_solve, lib.fvem_solve_adjoint):
        fn.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
        fn.restype = ctypes.c_int
    lib.fvem_apply.argtypes = [vp, i32, vp, vp, vp]
    lib.fvem_apply.restype = ctypes.c_int
    lib.fvem_project_velocity.argtypes = [vp, vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
    lib.fvem_project_velocity.restype = ctypes.c_int
    lib.fvem_project_velocity_adjoint.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats),
                                                  vp]
    lib.fvem_project_velocity_adjoint.restype = ctypes.c_int
    lib.fvem_velocity_loss.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp, vp]
    lib.fvem_velocity_loss.restype = ctypes.c_int
    lib.fvem_level_storage.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                       ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fvem_level_storage.restype = ctypes.c_int
    lib.fvem_level_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(i64)]
    lib.fvem_level_bytes.restype = ctypes.c_int
    lib.fvem_hierarchy_cells.argtypes = [vp, ctypes.POINTER(i64)]
    lib.fvem_hierarchy_cells.restype = ctypes.c_int
    lib.fvem_transfer_storage.argtypes = [vp, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                          ctypes.POINTER(i64)]
    lib.fvem_transfer_storage.restype = ctypes.c_int
    lib.fvem_memory_breakdown.argtypes = [vp, vp]
    lib.fvem_memory_breakdown.restype = ctypes.c_int
    lib.fvem_level_slices.argtypes = [vp, i32] + [ctypes.POINTER(i64)] * 4
    lib.fvem_level_slices.restype = ctypes.c_int
    lib.fvem_vcycle_bytes.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.fvem_vcycle_bytes.restype = ctypes.c_int
    lib.fvem_level_stencil.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.fvem_level_stencil.restype = ctypes.c_int
    lib.fvem_project_noalloc.argtypes = [vp, vp, vp, vp]
    lib.fvem_project_noalloc.restype = ctypes.c_int
    lib.fvem_level_matrix.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp]
    lib.fvem_level_matrix.restype = ctypes.c_int
    lib.fvem_hierarchy_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(i64)]
    lib.fvem_hierarchy_info.restype = ctypes.c_int
    lib.fvem_hierarchy_destroy.argtypes = [vp]
    lib.fvem_hierarchy_destroy.restype = None
    lib.fvem_last_error.argtypes = []
    lib.fvem_last_error.restype = ctypes.c_char_p
    lib.fvem_grid_build.argtypes = [vp, i64, vp, i64, i32, i32, i32, i32, i64, ctypes.POINTER(vp)]
    lib.fvem_grid_build.restype = ctypes.c_int
    lib.fvem_grid_build_ex.argtypes = [vp, i64, vp, i64, i32, i32, i32, i32, i64, i32, ctypes.POINTER(vp)]
    lib.fvem_grid_build_ex.restype = ctypes.c_int
    lib.fvem_grid_describe.argtypes = [vp, ctypes.POINTER(_Grid)]
    lib.fvem_grid_describe.restype = ctypes.c_int
    lib.fvem_grid_info.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                   ctypes.POINTER(i64)]
    lib.fvem_grid_info.restype = ctypes.c_int
    lib.fvem_grid_level_points.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.fvem_grid_level_points.restype = ctypes.c_int
    lib.fvem_grid_destroy.argtypes = [vp]
    lib.fvem_grid_destroy.restype = None
    lib.fvem_grid_cell_faces.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp, i32, i32]
    lib.fvem_grid_cell_faces.restype = ctypes.c_int
    lib.fvem_transport_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
    lib.fvem_transport_create.restype = ctypes.c_int
    lib.fvem_transport_destroy.argtypes = [vp]
    lib.fvem_transport_destroy.restype = None
    lib.fvem_locate.argtypes = [vp, i64, vp, vp, vp]
    lib.fvem_locate.restype = ctypes.c_int
    lib.fvem_p2g.argtypes = [vp, i64, vp, vp, i32, vp, vp]
    lib.fvem_p2g.restype = ctypes.c_int
    lib.fvem_buoyancy.argtypes = [vp, vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.fvem_buoyancy.restype = ctypes.c_int
    lib.fvem_g2p.argtypes = [vp, i64, vp, vp, vp, vp, vp, ctypes.c_double, vp]
    lib.fvem_g2p.restype = ctypes.c_int
    lib.fvem_advect.argtypes = [vp, i64, vp, vp, vp, ctypes.c_double, i32, ctypes.POINTER(i32), vp]
    lib.fvem_advect.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code):
    if code == 0:
        return
    msg = load().fvem_last_error().decode()
    if code == 5:
        raise NotConverged(code, msg)
    raise FvemError(code, msg)


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


class Hierarchy:
    """Solver hierarchy built from a problem description (host numpy arrays).

    ``desc`` keys: ``levels`` (list of dicts with n_dof, cell_ptr, cell_dof,
    parent, P given as (row_ptr, col, val) or None, and optionally
    dof_lattice [n_dof x 3] with lattice_n), ``ke_off``, ``ke_val``,
    ``n_vert``, ``cell_vptr``, ``cell_vert``, ``be_off``, ``be_val``,
    ``component``, ``n_components``, and the optional velocity blocks
    ``vc_off``, ``vc_val``, ``cell_geom``, ``vert_xyz``.
    """

    def __init__(self, desc, stream=None, cheb_degree=5, cheb_lower=1.0 / 30.0, coarse_dense_max=16384,
                 coarse_rcond=0.0, coarse_shift=1e-8, small_level_rows=0, max_templates=0,
                 lattice_min_fraction=0.0, galerkin_general=False, column_codes=0, vcycle_graphs=0):
        import torch
        lib = load()
        if not torch.cuda.is_available():
            raise FvemError(2, "no GPU visible")
        if isinstance(desc, Grid):
            g = _Grid()
            _check(lib.fvem_grid_describe(desc._g, ctypes.byref(g)))
            self._finish(lib, g, [desc], stream, cheb_degree, cheb_lower, coarse_dense_max, coarse_rcond,
                         coarse_shift, small_level_rows, max_templates, lattice_min_fraction, galerkin_general,
                         column_codes, vcycle_graphs)
            return
        keep = []
        L = len(desc["levels"])
        levels = (_Level * L)()
        for l, lv in enumerate(desc["levels"]):
            cp, cpp = _arr(lv["cell_ptr"], np.int64)
            cd, cdp = _arr(lv["cell_dof"], np.int32)
            keep += [cp, cd]
            levels[l].n_dof = int(lv["n_dof"])
            levels[l].n_cells = len(cp) - 1
            levels[l].cell_ptr = cpp
            levels[l].cell_dof = cdp
            if lv.get("parent") is not None:
                pa, pap = _arr(lv["parent"], np.int32)
                keep.append(pa)
                levels[l].parent = pap
            if lv.get("dof_lattice") is not None:
                la, lap = _arr(lv["dof_lattice"], np.int32)
                keep.append(la)
                levels[l].dof_lattice = lap
                levels[l].lattice_n = int(lv["lattice_n"])
            if lv.get("P") is not None:
                rp, ci, va = lv["P"]
                rp, rpp = _arr(rp, np.int64)
                ci, cip = _arr(ci, np.int32)
                va, vap = _arr(va, np.float64)
                keep += [rp, ci, va]
                levels[l].P = _CSR(len(rp) - 1, int(lv["P_cols"]), len(ci), rpp, cip, vap)
        g = _Grid()
        g.n_levels = L
        g.levels = levels
        for name, dt in (("ke_off", np.int64), ("ke_val", np.float64), ("cell_vptr", np.int64),
                         ("cell_vert", np.int32), ("be_off", np.int64), ("be_val", np.float64),
                         ("component", np.int32), ("vc_off", np.int64), ("vc_val", np.float64),
                         ("cell_geom", np.float64), ("vert_xyz", np.float64)):
            if desc.get(name) is not None:
                a, p = _arr(desc[name], dt)
                keep.append(a)
                setattr(g, name, p)
        g.ke_len = len(desc["ke_val"])
        g.be_len = len(desc["be_val"]) if desc.get("be_val") is not None else 0
        g.vc_len = len(desc["vc_val"]) if desc.get("vc_val") is not None else 0
        g.n_vert = int(desc.get("n_vert", 0))
        g.n_components = int(desc.get("n_components", 0))
        self._finish(lib, g, keep, stream, cheb_degree, cheb_lower, coarse_dense_max, coarse_rcond, coarse_shift,
                     small_level_rows, max_templates, lattice_min_fraction, galerkin_general, column_codes,
                     vcycle_graphs)

    def _finish(self, lib, g, keep, stream, cheb_degree, cheb_lower, coarse_dense_max, coarse_rcond, coarse_shift,
                small_level_rows, max_templates, lattice_min_fraction, galerkin_general, column_codes,
                vcycle_graphs):
        import torch
        opts = _Options(cheb_degree, cheb_lower, coarse_dense_max, coarse_rcond, coarse_shift, small_level_rows,
                        max_templates, lattice_min_fraction, int(column_codes), 1 if galerkin_general else 0,
                        int(vcycle_graphs))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib.fvem_hierarchy_build(ctypes.byref(g), ctypes.byref(opts), ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(h)))
        self._h = h
        nl, n0, nv, nb = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.fvem_hierarchy_info(h, ctypes.byref(nl), ctypes.byref(n0), ctypes.byref(nv), ctypes.byref(nb)))
        self.n_levels, self.n_dof, self.n_vert, self.device_bytes = nl.value, n0.value, nv.value, nb.value
        ncv = ctypes.c_int64()
        _check(lib.fvem_hierarchy_cells(h, ctypes.byref(ncv)))
        self.n_cells = ncv.value
        self.device = torch.device("cuda", torch.cuda.current_device())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fvem_hierarchy_destroy(h)
            self._h = None

    def _vec(self, t, n, what):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() \
                or t.device != self.device or t.numel() != n:
            raise ValueError(f"{what}: expected a contiguous float64 tensor of {n} elements on {self.device}")
        return ctypes.c_void_p(t.data_ptr())

    def _opts(self, tol, maxit, precision, input_kind, replace_every, profile):
        # profile: True or 1 times every V-cycle and finest-level launch (kernel by
        # kernel); 2 times only the V-cycles (graph replays stay on)
        return SolveOpts(tol, maxit, precision, input_kind, replace_every, int(profile) if profile else 0)

    def solve(self, inp, out=None, tol=1e-8, maxit=500, precision=PREC_MIXED, input_kind=INPUT_VELOCITY,
              replace_every=10, profile=False, raise_not_converged=True):
        import torch
        n_in = 3 * self.n_vert if input_kind == INPUT_VELOCITY else self.n_dof
        pin = self._vec(inp, n_in, "input")
        if out is None:
            out = torch.empty(self.n_dof, dtype=torch.float64, device=self.device)
        pout = self._vec(out, self.n_dof, "output")
        st = SolveStats()
        so = self._opts(tol, maxit, precision, input_kind, replace_every, profile)
        code = load().fvem_solve(self._h, pin, pout, ctypes.byref(so), ctypes.byref(st),
                                 ctypes.c_void_p(self.stream.cuda_stream))
        if code != 5 or raise_not_converged:
            _check(code)
        return out, st.as_dict()

    def solve_adjoint(self, gp, out=None, tol=1e-8, maxit=500, precision=PREC_MIXED, input_kind=INPUT_VELOCITY,
                      replace_every=10):
        import torch
        n_out = 3 * self.n_vert if input_kind == INPUT_VELOCITY else self.n_dof
        pin = self._vec(gp, self.n_dof, "g_p")
        if out is None:
            out = torch.empty(n_out, dtype=torch.float64, device=self.device)
        pout = self._vec(out, n_out, "output")
        st = SolveStats()
        so = self._opts(tol, maxit, precision, input_kind, replace_every, False)
        _check(load().fvem_solve_adjoint(self._h, pin, pout, ctypes.byref(so), ctypes.byref(st),
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        return out, st.as_dict()

    def _op_sizes(self, op):
        nv3, n, nc = 3 * self.n_vert, self.n_dof, 12 * self.n_cells
        return {OP_K: (n, n), OP_B: (nv3, n), OP_BT: (n, nv3), OP_VCYCLE: (n, n), OP_VCYCLE32: (n, n),
                OP_PROJECT: (n, n), OP_PI1: (nv3, nc), OP_PI1T: (nc, nv3), OP_G: (n, nc), OP_GT: (nc, n),
                OP_MASS: (nc, nc), OP_AV: (nc, nv3), OP_AVT: (nv3, nc)}[op]

    def apply(self, op, x, out=None, accumulate=False):
        """y = op(x), or out += op(x) with accumulate (velocity operators and B^T)."""
        import torch
        n_in, n_out = self._op_sizes(op)
        y = out if out is not None else torch.empty(n_out, dtype=torch.float64, device=self.device)
        code = op | (APPLY_ACCUMULATE if accumulate else 0)
        _check(load().fvem_apply(self._h, code, self._vec(x, n_in, "x"), self._vec(y, n_out, "y"),
                                 ctypes.c_void_p(self.stream.cuda_stream)))
        return y

    def project_noalloc(self, x, out=None):
        """y = P_perp x through fvem_project_noalloc (no allocation inside the library)."""
        import torch
        y = out if out is not None else torch.empty(self.n_dof, dtype=torch.float64, device=self.device)
        _check(load().fvem_project_noalloc(self._h, self._vec(x, self.n_dof, "x"), self._vec(y, self.n_dof, "y"),
                                           ctypes.c_void_p(self.stream.cuda_stream)))
        return y

    def project_velocity(self, u, s=None, p=None, tol=1e-8, maxit=500, precision=PREC_MIXED,
                         raise_not_converged=True):
        """Projected velocity s = Pi_1 u - grad Pi_k p (12 values per cell), with p = K^+ P B u."""
        import torch
        nc = 12 * self.n_cells
        if s is None:
            s = torch.empty(nc, dtype=torch.float64, device=self.device)
        pp = self._vec(p, self.n_dof, "p") if p is not None else None
        st = SolveStats()
        so = self._opts(tol, maxit, precision, INPUT_VELOCITY, 10, False)
        code = load().fvem_project_velocity(self._h, self._vec(u, 3 * self.n_vert, "u"), self._vec(s, nc, "s"), pp,
                                            ctypes.byref(so), ctypes.byref(st),
                                            ctypes.c_void_p(self.stream.cuda_stream))
        if code != 5 or raise_not_converged:
            _check(code)
        return s, st.as_dict()

    def project_velocity_adjoint(self, gs, gu=None, tol=1e-8, maxit=500, precision=PREC_MIXED):
        """g_u = Pi_1^T g_s + B^T P K^+ P (-(grad Pi_k)^T g_s), the transpose of u -> s."""
        import torch
        if gu is None:
            gu = torch.empty(3 * self.n_vert, dtype=torch.float64, device=self.device)
        st = SolveStats()
        so = self._opts(tol, maxit, precision, INPUT_VELOCITY, 10, False)
        _check(load().fvem_project_velocity_adjoint(self._h, self._vec(gs, 12 * self.n_cells, "g_s"),
                                                    self._vec(gu, 3 * self.n_vert, "g_u"), ctypes.byref(so),
                                                    ctypes.byref(st), ctypes.c_void_p(self.stream.cuda_stream)))
        return gu, st.as_dict()

    def velocity_loss(self, s, t, scale=1.0, grad=True):
        """(L, g_s): L = sum_E int_E |s - t|^2, g_s = scale * dL/ds (None without grad)."""
        import torch
        nc = 12 * self.n_cells
        gs = torch.empty(nc, dtype=torch.float64, device=self.device) if grad else None
        L = ctypes.c_double()
        _check(load().fvem_velocity_loss(self._h, self._vec(s, nc, "s"), self._vec(t, nc, "t"), float(scale),
                                         ctypes.byref(L), self._vec(gs, nc, "g_s") if grad else None,
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        return L.value, gs

    def level_storage(self, level):
        """Storage of level ``level``'s operator: nnz, nnz_explicit, rows_templated, n_templates, template_width."""
        v = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()]
        _check(load().fvem_level_storage(self._h, level, *[ctypes.byref(x) for x in v]))
        return dict(zip(("nnz", "nnz_explicit", "rows_templated", "n_templates", "template_width"),
                        (x.value for x in v)))

    def memory_breakdown(self):
        """Device bytes held by the handle, by structure (fvem_memory_breakdown)."""
        b = np.zeros(8, dtype=np.int64)
        _check(load().fvem_memory_breakdown(self._h, b.ctypes.data))
        return dict(zip(("level_operators", "transfers", "level_vectors", "divergence", "velocity_operators",
                         "coarsest_inverse", "cg_workspace", "total"), (int(v) for v in b)))

    def level_slices(self, level):
        """Slices of level ``level``'s sliced operator: coded, plain, templated, stored."""
        v = [ctypes.c_int64() for _ in range(4)]
        _check(load().fvem_level_slices(self._h, level, *[ctypes.byref(x) for x in v]))
        return dict(zip(("coded", "plain", "templated", "stored"), (x.value for x in v)))

    def transfer_storage(self, level, precision=PREC_MIXED):
        """P_level nonzeros and the matrix bytes of one application of P_level and R_level."""
        v = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()]
        _check(load().fvem_transfer_storage(self._h, level, precision, *[ctypes.byref(x) for x in v]))
        return dict(zip(("nnz", "bytes_p", "bytes_r"), (x.value for x in v)))

    def transfer_nnz(self, level):
        return self.transfer_storage(level)["nnz"]

    def vcycle_bytes(self, precision=PREC_MIXED):
        """Algorithmic bytes of one V-cycle (fvem_vcycle_bytes)."""
        b = ctypes.c_int64()
        _check(load().fvem_vcycle_bytes(self._h, precision, ctypes.byref(b)))
        return b.value

    def level_stencil(self, level):
        """Lattice stencil part of level ``level``'s operator: rows, nnz, tiles."""
        v = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()]
        _check(load().fvem_level_stencil(self._h, level, *[ctypes.byref(x) for x in v]))
        return dict(zip(("rows", "nnz", "tiles"), (x.value for x in v)))

    def level_bytes(self, level, precision=PREC_MIXED):
        """Matrix bytes one application of level ``level``'s operator reads (see fvem_level_bytes)."""
        b = ctypes.c_int64()
        _check(load().fvem_level_bytes(self._h, level, precision, ctypes.byref(b)))
        return b.value

    def level_rows(self, level):
        """DOFs (rows) of level ``level``'s operator."""
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        _check(load().fvem_level_matrix(self._h, level, ctypes.byref(n), ctypes.byref(nnz), None, None, None))
        return n.value

    def level_matrix(self, level):
        """Level operator as (row_ptr, col, val) host arrays."""
        lib = load()
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.fvem_level_matrix(self._h, level, ctypes.byref(n), ctypes.byref(nnz), None, None, None))
        rp = np.empty(n.value + 1, dtype=np.int64)
        ci = np.empty(nnz.value, dtype=np.int32)
        va = np.empty(nnz.value, dtype=np.float64)
        _check(lib.fvem_level_matrix(self._h, level, ctypes.byref(n), ctypes.byref(nnz), rp.ctypes.data,
                                     ci.ctypes.data, va.ctypes.data))
        return rp, ci, va


class Grid:
    """Native cut-cell grid, VEM operators and hierarchy built from a boundary mesh (host C++)."""

    def __init__(self, V, F, N, k, levels=5, dirichlet_top=False, coarse_max=16384, naive_prolongation=False):
        lib = load()
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        g = ctypes.c_void_p()
        _check(lib.fvem_grid_build_ex(V.ctypes.data, len(V), F.ctypes.data, len(F), int(N), int(k), int(levels),
                                      1 if dirichlet_top else 0, int(coarse_max),
                                      GRID_NAIVE_PROLONGATION if naive_prolongation else 0, ctypes.byref(g)))
        self._g = g
        self.N, self.k = N, k
        xv, nv, dp, dk = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_void_p(), ctypes.c_void_p()
        nd, ntr, nsh = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.fvem_grid_info(g, ctypes.byref(xv), ctypes.byref(nv), ctypes.byref(dp), ctypes.byref(dk),
                                  ctypes.byref(nd), ctypes.byref(ntr), ctypes.byref(nsh)))
        self.n_vert, self.n_dof, self.n_trees, self.n_shared_blocks = nv.value, nd.value, ntr.value, nsh.value
        self.vertices = np.ctypeslib.as_array(ctypes.cast(xv, ctypes.POINTER(ctypes.c_double)),
                                              shape=(self.n_vert, 3)).copy()
        self.dof_points = np.ctypeslib.as_array(ctypes.cast(dp, ctypes.POINTER(ctypes.c_double)),
                                                shape=(self.n_dof, 3)).copy()
        self.dof_kind = np.ctypeslib.as_array(ctypes.cast(dk, ctypes.POINTER(ctypes.c_int8)),
                                              shape=(self.n_dof,)).copy()

    def cell_faces(self, cell):
        """Outward vertex cycles (arrays of vertex ids) of finest-level cell ``cell``."""
        lib = load()
        nf, nc = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.fvem_grid_cell_faces(self._g, int(cell), ctypes.byref(nf), ctypes.byref(nc), None, None, 0, 0))
        lens = np.zeros(nf.value, dtype=np.int32)
        verts = np.zeros(nc.value, dtype=np.int32)
        _check(lib.fvem_grid_cell_faces(self._g, int(cell), None, None, lens.ctypes.data, verts.ctypes.data,
                                        nf.value, nc.value))
        return np.split(verts, np.cumsum(lens)[:-1])

    def level_points(self, level):
        """(points [n x 3], kinds [n]) of level ``level``'s free DOFs."""
        lib = load()
        dp, dk, n = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        _check(lib.fvem_grid_level_points(self._g, level, ctypes.byref(dp), ctypes.byref(dk), ctypes.byref(n)))
        if n.value == 0:
            return np.zeros((0, 3)), np.zeros(0, dtype=np.int8)
        pts = np.ctypeslib.as_array(ctypes.cast(dp, ctypes.POINTER(ctypes.c_double)), shape=(n.value, 3)).copy()
        knd = np.ctypeslib.as_array(ctypes.cast(dk, ctypes.POINTER(ctypes.c_int8)), shape=(n.value,)).copy()
        return pts, knd

    def describe(self):
        """The problem description as host numpy arrays (copies)."""
        lib = load()
        g = _Grid()
        _check(lib.fvem_grid_describe(self._g, ctypes.byref(g)))

        def arr(ptr, n, ct):
            if n == 0:
                return np.zeros(0, dtype=np.ctypeslib.as_array((ct * 1)()).dtype)
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(n,)).copy()

        levels = []
        for l in range(g.n_levels):
            lv = g.levels[l]
            cp = arr(lv.cell_ptr, lv.n_cells + 1, ctypes.c_int64)
            d = {"n_dof": lv.n_dof, "cell_ptr": cp, "cell_dof": arr(lv.cell_dof, int(cp[-1]), ctypes.c_int32),
                 "parent": None, "P": None,
                 "dof_lattice": arr(lv.dof_lattice, 3 * lv.n_dof, ctypes.c_int32) if lv.dof_lattice else None,
                 "lattice_n": lv.lattice_n}
            if l + 1 < g.n_levels:
                d["parent"] = arr(lv.parent, lv.n_cells, ctypes.c_int32)
                P = lv.P
                d["P"] = (arr(P.row_ptr, P.n_rows + 1, ctypes.c_int64), arr(P.col, P.nnz, ctypes.c_int32),
                          arr(P.val, P.nnz, ctypes.c_double))
                d["P_cols"] = P.n_cols
            levels.append(d)
        nc0 = g.levels[0].n_cells
        vptr = arr(g.cell_vptr, nc0 + 1, ctypes.c_int64)
        return {"levels": levels, "ke_off": arr(g.ke_off, nc0, ctypes.c_int64),
                "ke_val": arr(g.ke_val, g.ke_len, ctypes.c_double), "n_vert": g.n_vert, "cell_vptr": vptr,
                "cell_vert": arr(g.cell_vert, int(vptr[-1]), ctypes.c_int32),
                "be_off": arr(g.be_off, nc0, ctypes.c_int64), "be_val": arr(g.be_val, g.be_len, ctypes.c_double),
                "component": arr(g.component, g.levels[0].n_dof, ctypes.c_int32),
                "n_components": g.n_components,
                "vc_off": arr(g.vc_off, nc0, ctypes.c_int64), "vc_val": arr(g.vc_val, g.vc_len, ctypes.c_double),
                "cell_geom": arr(g.cell_geom, 5 * nc0, ctypes.c_double),
                "vert_xyz": arr(g.vert_xyz, 3 * g.n_vert, ctypes.c_double)}

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and _lib is not None:
            _lib.fvem_grid_destroy(g)
            self._g = None


def project_function():
    """torch.autograd.Function mapping vertex velocity u -> pressure p.

    forward: p = K^+ P_perp B u (fvem_solve); backward: g_u = B^T P_perp K^+
    P_perp g_p (fvem_solve_adjoint, the transpose of the linear map).
    """
    import torch

    class FvemProject(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u, hier, tol, precision):
            ctx.hier, ctx.tol, ctx.precision = hier, tol, precision
            p, _ = hier.solve(u.contiguous(), tol=tol, precision=precision)
            return p

        @staticmethod
        def backward(ctx, gp):
            gu, _ = ctx.hier.solve_adjoint(gp.contiguous(), tol=ctx.tol, precision=ctx.precision)
            return gu, None, None, None

    return FvemProject


def velocity_function():
    """torch.autograd.Function mapping vertex velocity u -> projected cell field s.

    forward: s = Pi_1 u - grad Pi_k K^+ P B u (fvem_project_velocity);
    backward: the transpose (fvem_project_velocity_adjoint).  The map is
    linear, so nothing of the forward pass is saved.
    """
    import torch

    class FvemVelocity(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u, hier, tol, precision):
            ctx.hier, ctx.tol, ctx.precision = hier, tol, precision
            s, _ = hier.project_velocity(u.contiguous(), tol=tol, precision=precision)
            return s

        @staticmethod
        def backward(ctx, gs):
            gu, _ = ctx.hier.project_velocity_adjoint(gs.contiguous(), tol=ctx.tol, precision=ctx.precision)
            return gu, None, None, None

    return FvemVelocity


def loss_function():
    """torch.autograd.Function (s, t) -> sum_E int_E |s_E - t_E|^2 (t is a constant target)."""
    import torch

    class FvemLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, s, t, hier):
            ctx.hier = hier
            ctx.save_for_backward(s, t)
            L, _ = hier.velocity_loss(s.contiguous(), t.contiguous(), grad=False)
            return torch.tensor(L, dtype=torch.float64, device=s.device)

        @staticmethod
        def backward(ctx, gL):
            s, t = ctx.saved_tensors
            _, gs = ctx.hier.velocity_loss(s, t, scale=float(gL), grad=True)
            return gs, None, None

    return FvemLoss


def chain_loss_and_grad(hier, u0, eps, targets, store_dtype=None, tol=1e-10, precision=PREC_MIXED, with_grad=True):
    """Loss of len(targets) chained projections and its gradient with respect to u0.

    Step k projects u_k to s_k, adds loss(s_k, t_k) and (except after the
    last step) moves on to u_{k+1} = Av s_k + eps_k.  Each step keeps one
    checkpoint, u_k stored in ``store_dtype`` (torch.float32 or
    torch.float64); the backward sweep re-runs that step's forward solve from
    the checkpoint, then its adjoint solve.  Returns (loss, grad, stats);
    grad is None without with_grad.
    """
    import torch
    store_dtype = store_dtype or torch.float64
    K = len(targets)
    ckpt = []
    total = 0.0
    u = u0.contiguous()
    for k in range(K):
        ckpt.append(u.to(store_dtype).clone())
        s, _ = hier.project_velocity(u, tol=tol, precision=precision)
        L, _ = hier.velocity_loss(s, targets[k], grad=False)
        total += L
        if k + 1 < K:
            u = eps[k].to(torch.float64).clone()
            hier.apply(OP_AV, s, out=u, accumulate=True)
    gu_next = None
    peak = sum(c.numel() * c.element_size() for c in ckpt)
    if not with_grad:
        return total, None, {"checkpoint_bytes": peak, "steps": K}
    for k in reversed(range(K)):
        uk = ckpt[k].to(torch.float64).contiguous()
        s, _ = hier.project_velocity(uk, tol=tol, precision=precision)
        _, gs = hier.velocity_loss(s, targets[k], grad=True)
        if gu_next is not None:
            hier.apply(OP_AVT, gu_next, out=gs, accumulate=True)
        gu_next, _ = hier.project_velocity_adjoint(gs, tol=tol, precision=precision)
    return total, gu_next, {"checkpoint_bytes": peak, "steps": K}


class Transport:
    """P2G, buoyancy, G2P and advection on a native grid's finest level
    (the steps around the solve in Algorithm 1).  Arrays are float64 (ghost
    flags uint8, cells int32) contiguous tensors on the current device."""

    def __init__(self, grid, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise FvemError(2, "no GPU visible")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.n_vert = grid.n_vert
        t = ctypes.c_void_p()
        _check(load().fvem_transport_create(grid._g, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(t)))
        self._t = t

    def __del__(self):
        t = getattr(self, "_t", None)
        if t is not None and _lib is not None:
            _lib.fvem_transport_destroy(t)
            self._t = None

    def _arr(self, a, shape, dtype, what):
        import torch
        if not isinstance(a, torch.Tensor) or a.dtype != dtype or a.device != self.device or \
                not a.is_contiguous() or tuple(a.shape) != tuple(shape):
            raise ValueError(f"{what}: expected a contiguous {dtype} tensor of shape {tuple(shape)} on {self.device}")
        return ctypes.c_void_p(a.data_ptr())

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def locate(self, x):
        import torch
        n = x.shape[0]
        cell = torch.empty(n, dtype=torch.int32, device=self.device)
        _check(load().fvem_locate(self._t, n, self._arr(x, (n, 3), torch.float64, "x"),
                                  self._arr(cell, (n,), torch.int32, "cell"), self._s()))
        return cell

    def p2g(self, x, f):
        import torch
        n, m = f.shape
        out = torch.empty((self.n_vert, m), dtype=torch.float64, device=self.device)
        _check(load().fvem_p2g(self._t, n, self._arr(x, (n, 3), torch.float64, "x"),
                               self._arr(f, (n, m), torch.float64, "f"), m,
                               self._arr(out, (self.n_vert, m), torch.float64, "out"), self._s()))
        return out

    def buoyancy(self, f, alpha, beta, dt):
        import torch
        m = f.shape[1]
        u = torch.empty(3 * self.n_vert, dtype=torch.float64, device=self.device)
        _check(load().fvem_buoyancy(self._t, self._arr(f, (self.n_vert, m), torch.float64, "f"), m, float(alpha),
                                    float(beta), float(dt), self._arr(u, (3 * self.n_vert,), torch.float64, "u"),
                                    self._s()))
        return u

    def g2p(self, x, ghost, u, s_new, s_old, a_flip):
        import torch
        n = x.shape[0]
        nc = s_new.shape[0]
        _check(load().fvem_g2p(self._t, n, self._arr(x, (n, 3), torch.float64, "x"),
                               self._arr(ghost, (n,), torch.uint8, "ghost"), self._arr(u, (n, 3), torch.float64, "u"),
                               self._arr(s_new, (nc,), torch.float64, "s_new"),
                               self._arr(s_old, (nc,), torch.float64, "s_old"), float(a_flip), self._s()))
        return u

    def advect(self, x, ghost, s, dt, max_substeps=64):
        import torch
        n = x.shape[0]
        sub = ctypes.c_int32()
        _check(load().fvem_advect(self._t, n, self._arr(x, (n, 3), torch.float64, "x"),
                                  self._arr(ghost, (n,), torch.uint8, "ghost"),
                                  self._arr(s, (s.shape[0],), torch.float64, "s"), float(dt), int(max_substeps),
                                  ctypes.byref(sub), self._s()))
        return x, sub.value


def smoke_step(hier, transport, x, u, rho, temp, ghost, dt, a_flip=0.95, alpha=0.0, beta=1.0, tol=1e-8,
               precision=PREC_MIXED):
    """One simulation step of Algorithm 1 on the GPU: P2G, buoyancy, the
    projection, G2P and advection.  x and u ([n, 3]) are updated in place;
    rho, temp ([n]) ride with the particles.  Each step is one library call;
    this function only sequences them."""
    import torch
    f = torch.cat([u, rho[:, None], temp[:, None]], dim=1).contiguous()
    fv = transport.p2g(x, f)
    u_grid = fv[:, :3].contiguous().view(-1)
    u_forced = transport.buoyancy(fv, alpha, beta, dt)
    s_new, st = hier.project_velocity(u_forced, tol=tol, precision=precision)
    s_old = hier.apply(OP_PI1, u_grid)
    transport.g2p(x, ghost, u, s_new, s_old, a_flip)
    _, n_sub = transport.advect(x, ghost, s_new, dt)
    return {"vertex": fv, "u_forced": u_forced, "s_new": s_new, "s_old": s_old, "substeps": n_sub,
            "iterations": st["iterations"]}
