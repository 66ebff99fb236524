/*
 * fvem.h - C ABI of the FastVEM pressure-projection solver for MI355X (gfx950).
 *
 * The library solves the pressure system of the paper's VEM projection
 * (Sec. 3.1: assemble K and r, solve K p = r; Sec. 3.2: r is the projected
 * divergence of the first-order vertex velocity) with CG preconditioned by
 * the paper's Galerkin geometric multigrid (Sec. 4: diffusion-free
 * prolongation P, restriction R = P^T, coarse operators A_c = R A_f P).
 *
 * Conventions for every entry point:
 *  - Every call returns an fvem_status and never throws across the ABI;
 *    fvem_last_error() returns a thread-local message for the last failure.
 *  - Host arrays passed in descriptors are owned by the caller and only read
 *    during the call; the library keeps copies.
 *  - Device pointers are HIP device memory on the device that was current
 *    when the hierarchy was built; work is enqueued on the given stream
 *    (NULL = the default stream) and is complete in stream order when the
 *    call returns.
 *  - Results are bitwise deterministic for a given input and build.
 *
 * The coarsest level of the hierarchy is solved with a dense Cholesky
 * factorisation of A_c + shift diag(A_c) (the paper does not specify the
 * coarse solver).  A_c is only positive semi-definite (pure-Neumann
 * constants; coarse DOF combinations the prolongation annihilates); every
 * right-hand side the V-cycle restricts to that level is orthogonal to those
 * directions, and what the shift adds along them vanishes after
 * prolongation.
 */
#ifndef FVEM_H
#define FVEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FVEM_OK = 0,
    FVEM_ERR_INVALID = 1,        /* malformed descriptor or argument */
    FVEM_ERR_HIP = 2,            /* a HIP runtime call failed; destroy the handle */
    FVEM_ERR_OOM = 3,            /* device or host allocation failed */
    FVEM_ERR_NOT_SPD = 4,        /* coarsest operator has a negative pivot */
    FVEM_ERR_NOT_CONVERGED = 5,  /* maxit reached; outputs hold the last iterate */
    FVEM_ERR_NONFINITE = 6,      /* NaN/Inf in the input or a CG breakdown */
    FVEM_ERR_BUSY = 7            /* another solve is running on this handle */
} fvem_status;

/* Compressed sparse rows.  row_ptr has n_rows+1 entries (int64), col holds
 * int32 column indices sorted within each row, val the FP64 values. */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
} fvem_csr;

/* One level of the nested hierarchy (level 0 = finest).
 *  n_dof     free (unknown) DOFs of the level.
 *  n_cells   cells of the level; cell c owns local DOFs
 *            cell_dof[cell_ptr[c] .. cell_ptr[c+1]), each a free DOF index or
 *            -1 for an eliminated DOF (Dirichlet, or a coarse DOF the
 *            prolongation never uses).  Local order: vertices, edges, faces,
 *            cell (Sec. 3.1 DOF list).
 *  parent    [n_cells] index of the cell of level+1 containing each cell
 *            (the hierarchy is nested, Sec. 5.2); NULL on the coarsest level.
 *  P         prolongation from level+1 to this level, n_dof x n_dof(level+1),
 *            diffusion-free: every row of a DOF of cell c may only reference
 *            DOFs of cell parent[c] (Sec. 4); unused on the coarsest level.
 *  dof_lattice optional [n_dof x 3]: integer coordinates of each DOF's
 *            support point on the level's structured lattice (cells of
 *            side 2^level h; the half-lattice of spacing 2^(level-1) h for
 *            k = 2, the vertex lattice for k = 1), or -1 where the point is
 *            off the lattice.  With it, rows that equal their lattice
 *            class's stencil are applied without stored columns or values
 *            (the compact storage of regular-grid regions that Sec. 7
 *            suggests); NULL keeps every row in sliced storage.
 *  lattice_n lattice points per axis (2 N / 2^level + 1 for k = 2,
 *            N / 2^level + 1 for k = 1). */
typedef struct {
    int64_t n_dof;
    int64_t n_cells;
    const int64_t *cell_ptr;
    const int32_t *cell_dof;
    const int32_t *parent;
    fvem_csr P;
    const int32_t *dof_lattice;
    int32_t lattice_n;
} fvem_level_desc;

/* The problem: hierarchy plus the finest level's element operators.
 *  ke_off/ke_val  element stiffness K^E of each level-0 cell, row-major
 *                 n_E x n_E over the cell's local DOFs (n_E = cell_ptr[c+1]
 *                 - cell_ptr[c]), starting at ke_val[ke_off[c]]; cells of
 *                 identical shape may share one block; ke_len is the length
 *                 of ke_val.
 *  n_vert, cell_vptr/cell_vert  velocity vertices; cell c's vertices are
 *                 cell_vert[cell_vptr[c] .. cell_vptr[c+1]).
 *  be_off/be_val  divergence block B^E of each cell, row-major
 *                 n_E x (3 n_vE) at be_val[be_off[c]]: column 3 v + d is
 *                 component d of the cell's v-th vertex velocity (Sec. 3.2
 *                 right-hand side); be_len is the length of be_val.
 *  component      [n_dof of level 0]: id of the pure-Neumann component of
 *                 each free DOF (0 .. n_components-1), or -1 where the
 *                 component is anchored by Dirichlet DOFs.
 *  vc_off/vc_val  optional velocity-correction block of each level-0 cell
 *                 (NULL: the velocity operators below are unavailable), at
 *                 vc_val[vc_off[c]], row-major, on the scaled linear
 *                 monomials z = [1, (x - x_E)/h_E] of App. A:
 *                   Pi1 (4 x n_vE): one velocity component's vertex values ->
 *                       coefficients of its linear projection Pi_1;
 *                   Gk (3 x 4 x n_E): pressure DOFs -> coefficients of
 *                       d/dx_c of Pi_k p, c = 0..2 (Sec. 3.3 correction);
 *                   M1 (4 x 4): int_E z z^T;
 *                 cells of identical shape may share a block; vc_len is the
 *                 length of vc_val.
 *  cell_geom      [n_cells x 5] centroid x_E, h_E (diameter) and volume of
 *                 each level-0 cell (with vc_off).
 *  vert_xyz       [n_vert x 3] velocity vertex coordinates (with vc_off). */
typedef struct {
    int32_t n_levels;
    const fvem_level_desc *levels;
    const int64_t *ke_off;
    const double *ke_val;
    int64_t ke_len;
    int64_t n_vert;
    const int64_t *cell_vptr;
    const int32_t *cell_vert;
    const int64_t *be_off;
    const double *be_val;
    int64_t be_len;
    const int32_t *component;
    int32_t n_components;
    const int64_t *vc_off;
    const double *vc_val;
    int64_t vc_len;
    const double *cell_geom;
    const double *vert_xyz;
} fvem_grid_desc;

/* Hierarchy options.  Zero-initialised fields take the defaults in brackets. */
typedef struct {
    int32_t cheb_degree;        /* Chebyshev degree per smoothing [5] */
    double cheb_lower;          /* lower end of the interval as a fraction of lmax [1/30] */
    int32_t coarse_dense_max;   /* largest coarsest level factored densely [16384] */
    double coarse_rcond;        /* pivots below rcond * diag are treated as zero [0] */
    double coarse_shift;        /* the coarsest level factors A_c + shift diag(A_c) [1e-8] */
    int64_t small_level_rows;   /* levels (or the sliced rows of a lattice level) with at most
                                   this many rows share each row among 16 lanes instead of one
                                   lane per row [400000]; < 0: never */
    int32_t max_templates;      /* value templates per operator [4096]; < 0: none */
    double lattice_min_fraction; /* with dof_lattice: use the lattice stencil layout on a level
                                    below the coarsest when at least this fraction of its rows
                                    are stencil rows [0.5]; < 0: never */
    int32_t column_codes;       /* 0: 16-bit column codes for every slice whose columns allow
                                   them [default]; < 0: int32 columns everywhere */
    int32_t galerkin_general;   /* nonzero: form every coarse operator as P^T A P by sparse
                                   products on the host, for prolongations whose rows reach
                                   beyond one coarse cell (the naive prolongation of Sec. 4);
                                   0: the element-wise product, which requires the
                                   diffusion-free structure [0] */
    int32_t vcycle_graphs;      /* 0: replay each V-cycle as a HIP graph, captured at its first
                                   use on a stream the hierarchy owns and joined to the caller's
                                   stream by events [default]; < 0: launch its kernels one by
                                   one on the caller's stream (profiled solves always do) */
} fvem_options;

typedef enum { FVEM_PREC_FP64 = 0, FVEM_PREC_MIXED = 1 } fvem_precision;
typedef enum { FVEM_INPUT_VELOCITY = 0, FVEM_INPUT_RHS = 1 } fvem_input;

typedef struct {
    double tol;             /* stop when ||b - K x|| / ||b|| <= tol [1e-8] */
    int32_t maxit;          /* [500] */
    int32_t precision;      /* fvem_precision: FP32 V-cycle inside FP64 CG, or all FP64 */
    int32_t input;          /* fvem_input */
    int32_t replace_every;  /* true-residual replacement period [10] */
    int32_t profile;        /* 1: time every V-cycle and every finest-level Chebyshev launch
                               (HIP events; V-cycles then launch kernel by kernel); 2: time
                               only the V-cycles (graph replays stay on); 0: no timing */
} fvem_solve_opts;

typedef struct {
    int32_t iterations;
    double rel_residual;    /* true ||b - K x|| / ||b|| at exit (FP64) */
    double ms_total;        /* device time of the call (HIP events) */
    double ms_fine_smoother; /* with profile: summed device time of the finest-level
                                fused Chebyshev-step launches (SpMV + update) */
    int32_t n_fine_smoother; /* with profile: number of those launches */
    int32_t n_levels;
    double ms_vcycle;       /* with profile: summed device time of the preconditioner's V-cycles */
    int32_t n_vcycle;       /* with profile: number of those V-cycles */
    double ms_fine_stencil; /* with profile: summed device time of the lattice stencil launches
                               inside the finest-level Chebyshev steps (0 without stencil rows) */
    int32_t n_fine_stencil; /* with profile: number of those launches */
} fvem_solve_stats;

typedef struct fvem_hierarchy fvem_hierarchy;

/* Build the solver hierarchy on the current device (setup, Sec. 4).
 * Assembles K from the element blocks, forms A_{l+1} = P_l^T A_l P_l
 * element-wise per coarse cell, transposes P, computes Chebyshev bounds,
 * FP32 copies and the coarsest-level factorisation, and preallocates every
 * solve buffer.  Where a coarse level below the coarsest gives dof_lattice,
 * the element blocks of translated copies of a lattice-aligned coarse cell
 * that agree to 1e-12 of their largest entry (rounding of the product) are
 * replaced by the first such block, so that translated rows are equal and
 * can be applied as lattice stencils.  Errors: INVALID (bad sizes, indices out of range, a P row
 * that references a DOF outside its cell's parent, non-finite values), OOM,
 * HIP, NOT_SPD.  On success *out owns all device memory. */
fvem_status fvem_hierarchy_build(const fvem_grid_desc *g, const fvem_options *o,
                                 void *hip_stream, fvem_hierarchy **out);

/* Pressure solve.  in_dev: velocity [3 n_vert] (FVEM_INPUT_VELOCITY, b = B u)
 * or right-hand side [n_dof0] (FVEM_INPUT_RHS).  p_dev: [n_dof0] output,
 * zero DOF mean on every pure-Neumann component.  Returns NOT_CONVERGED
 * (outputs and stats still written) when maxit is reached. */
fvem_status fvem_solve(fvem_hierarchy *h, const double *in_dev, double *p_dev,
                       const fvem_solve_opts *so, fvem_solve_stats *st, void *hip_stream);

/* Adjoint of fvem_solve: given g_p [n_dof0], returns
 * g_u = B^T P_perp K^+ P_perp g_p [3 n_vert] (FVEM_INPUT_VELOCITY) or
 * g_b = P_perp K^+ P_perp g_p [n_dof0] (FVEM_INPUT_RHS).  K is symmetric
 * (Sec. 3.1), so the same MG-PCG and hierarchy solve the adjoint system. */
fvem_status fvem_solve_adjoint(fvem_hierarchy *h, const double *gp_dev, double *gu_dev,
                               const fvem_solve_opts *so, fvem_solve_stats *st, void *hip_stream);

/* Operators used by tests and loss plumbing (all FP64, device vectors). */
typedef enum {
    FVEM_OP_K = 0,        /* y[n_dof0] = K x[n_dof0] */
    FVEM_OP_B = 1,        /* y[n_dof0] = B x[3 n_vert] */
    FVEM_OP_BT = 2,       /* y[3 n_vert] = B^T x[n_dof0] */
    FVEM_OP_VCYCLE = 3,   /* y[n_dof0] = M x: one V-cycle of the preconditioner (FP64) */
    FVEM_OP_VCYCLE32 = 4, /* the same V-cycle with FP32 smoothing and transfers */
    FVEM_OP_PROJECT = 5,  /* y = P_perp x (zero mean per pure-Neumann component) */
    /* velocity operators (need vc_off at build).  A cell field holds 12
     * values per level-0 cell, ordered (cell, component c, coefficient a) on
     * the monomials z of vc_val. */
    FVEM_OP_PI1 = 6,      /* y[12 n_cells] = Pi_1 x[3 n_vert] */
    FVEM_OP_PI1T = 7,     /* y[3 n_vert] = Pi_1^T x[12 n_cells] */
    FVEM_OP_G = 8,        /* y[12 n_cells] = grad Pi_k x[n_dof0] */
    FVEM_OP_GT = 9,       /* y[n_dof0] = (grad Pi_k)^T x[12 n_cells] */
    FVEM_OP_MASS = 10,    /* y[12 n_cells] = blockdiag(M1) x[12 n_cells] */
    FVEM_OP_AV = 11,      /* y[3 n_vert] = Av x[12 n_cells]: each vertex gets the
                             volume-weighted mean of its cells' fields at the vertex */
    FVEM_OP_AVT = 12      /* y[12 n_cells] = Av^T x[3 n_vert] */
} fvem_op;

/* op | FVEM_APPLY_ACCUMULATE adds to y instead of overwriting it (all ops
 * but VCYCLE, VCYCLE32 and PROJECT). */
#define FVEM_APPLY_ACCUMULATE 0x100

fvem_status fvem_apply(fvem_hierarchy *h, int32_t op, const double *x_dev, double *y_dev,
                       void *hip_stream);

/* Projected velocity (Sec. 3.3 correction after the Sec. 3.1 solve):
 * p = fvem_solve(u), s = Pi_1 u - grad Pi_k p.  u_dev [3 n_vert], s_dev
 * [12 n_cells]; p_dev [n_dof0] receives the pressure unless NULL.  Same
 * options, stats, errors and stream rules as fvem_solve; needs vc_off. */
fvem_status fvem_project_velocity(fvem_hierarchy *h, const double *u_dev, double *s_dev, double *p_dev,
                                  const fvem_solve_opts *so, fvem_solve_stats *st, void *hip_stream);

/* Transpose of u -> s: g_u = Pi_1^T g_s + B^T P_perp K^+ P_perp (-(grad Pi_k)^T g_s).
 * gs_dev [12 n_cells], gu_dev [3 n_vert]. */
fvem_status fvem_project_velocity_adjoint(fvem_hierarchy *h, const double *gs_dev, double *gu_dev,
                                          const fvem_solve_opts *so, fvem_solve_stats *st,
                                          void *hip_stream);

/* Loss of a cell field against a target: L = sum_E int_E |s_E - t_E|^2
 * = (s - t)^T blockdiag(M1) (s - t), written to *loss_host (host memory);
 * when gs_dev is not NULL it receives scale * dL/ds = 2 scale M1 (s - t).
 * Deterministic (fixed-order reduction); synchronises the stream. */
fvem_status fvem_velocity_loss(fvem_hierarchy *h, const double *s_dev, const double *t_dev, double scale,
                               double *loss_host, double *gs_dev, void *hip_stream);

/* The component projection y = P_perp x of FVEM_OP_PROJECT (zero DOF mean on
 * every pure-Neumann component, caller's DOF order), for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It allocates nothing, creates no event
 * and does not synchronise: its reduction scratch is a static device array of
 * the library (about 256 KiB per device, taken when the first hierarchy is
 * built on that device), so it serves handles with at most 16 pure-Neumann
 * components (INVALID otherwise).  Every call on one device shares that
 * array: calls that overlap on one device (different streams or threads)
 * race.  x and y are [n_dof0] device vectors; y may equal x.  The result is
 * complete in stream order; it equals FVEM_OP_PROJECT's up to the rounding
 * of the per-component means. */
fvem_status fvem_project_noalloc(fvem_hierarchy *h, const double *x_dev, double *y_dev, void *hip_stream);

/* Level data for inspection: copies level l's operator A_l (FP64 CSR as
 * built on the device) to caller-owned host arrays.  Call first with NULL
 * arrays to get n_rows and nnz; then row_ptr needs n_rows+1, col/val nnz. */
fvem_status fvem_level_matrix(fvem_hierarchy *h, int32_t level, int64_t *n_rows, int64_t *nnz,
                              int64_t *row_ptr, int32_t *col, double *val);

/* Sizes: number of levels, and n_dof / nnz of level l. */
fvem_status fvem_hierarchy_info(fvem_hierarchy *h, int32_t *n_levels, int64_t *n_dof0,
                                int64_t *n_vert, int64_t *device_bytes);

/* Storage of level l's operator: nonzeros, nonzeros whose values are stored
 * with their slice, rows whose values come from the shared value templates
 * (their slices store columns only), number of templates and their width.
 * (FP32 value set; fvem_level_bytes gives the bytes one application reads). */
fvem_status fvem_level_storage(fvem_hierarchy *h, int32_t level, int64_t *nnz, int64_t *nnz_explicit,
                               int64_t *rows_templated, int32_t *n_templates, int32_t *template_width);

/* Device memory the handle holds, by structure: bytes[0] level operators
 * (sliced storage, templates, stencil tables), [1] transfers P_l and R_l,
 * [2] level vectors and inverse diagonals, [3] divergence B and B^T, [4]
 * velocity operators, [5] coarsest inverse, [6] CG workspace and the rest
 * allocated after the coarsest factorisation, [7] the total (bytes needs 8
 * entries). */
fvem_status fvem_memory_breakdown(fvem_hierarchy *h, int64_t *bytes);

/* Slices of level l's sliced operator by storage kind (FP32 value set):
 * with 16-bit column codes, with int32 columns, whose rows all read value
 * templates, and that store values. */
fvem_status fvem_level_slices(fvem_hierarchy *h, int32_t level, int64_t *coded, int64_t *plain,
                              int64_t *templated, int64_t *stored);

/* Matrix bytes one application of A_l reads in the given precision
 * (fvem_precision: FP64 or MIXED = FP32 values): 2 bytes per nonzero of
 * slices with 16-bit column codes plus 256 per block table, 4 per nonzero
 * of the others, the stored values (4 or 8 bytes per nonzero of
 * value-storing rows) and 4 per row reading a value template, 4 per row of a
 * row map (sliced rows scattered into the lattice layout) and 68 per tile of
 * lattice stencil rows (tile id and mask).  Padding and the cache-resident
 * template and stencil tables are not counted. */
fvem_status fvem_level_bytes(fvem_hierarchy *h, int32_t level, int32_t precision, int64_t *bytes);

/* Transfers between levels l and l+1: nonzeros of P_l and the matrix bytes
 * one application of P_l and of R_l = P_l^T reads in the given precision
 * (as fvem_level_bytes, plus 4 bytes per row of the row map). */
fvem_status fvem_transfer_storage(fvem_hierarchy *h, int32_t level, int32_t precision, int64_t *nnz,
                                  int64_t *bytes_p, int64_t *bytes_r);

/* Algorithmic bytes of one V-cycle of the preconditioner in the given
 * precision: on every level but the coarsest, 2 deg applications of A_l
 * (matrix bytes as fvem_level_bytes), one restriction and one
 * prolongation, and the vector streams of the fused kernels (per row: 4 for
 * the first smoothing step, 6 per later step, 3 for the residual, 1 for the
 * restriction, 2 for the correction, plus 2 per coarse row); on the
 * coarsest level the dense inverse (8 n_c^2) and its vectors.  Cache reuse
 * of gathered x is assumed; padding is not counted. */
fvem_status fvem_vcycle_bytes(fvem_hierarchy *h, int32_t precision, int64_t *bytes);

/* Lattice stencil part of level l's operator: rows applied from the class
 * stencils (no stored columns or values), their nonzeros, and the lattice
 * tiles launched per application (all zero when the level has none). */
fvem_status fvem_level_stencil(fvem_hierarchy *h, int32_t level, int64_t *rows, int64_t *nnz, int64_t *tiles);

/* Number of level-0 cells carrying velocity fields (0 without vc_off). */
fvem_status fvem_hierarchy_cells(fvem_hierarchy *h, int64_t *n_cells);

void fvem_hierarchy_destroy(fvem_hierarchy *h);

/* ---------------------------------------------------------------- grid builder
 * Builds the problem description from a boundary triangle mesh (host, C++):
 * the binary-space cut-cell grid of Sec. 5.1 (each background cell split by
 * the planes of its triangles, fewest plane crossings first; parts below
 * 1e-12 volume skipped; leaves classified interior/exterior), the nested
 * boundary-aware hierarchy of Sec. 5.2 (aggregation of uncut cubes, greedy
 * removal of least-important cuts up to 1/L of the weight per level), the
 * conforming order-k VEM element operators of Sec. 3.1-3.2 and the
 * diffusion-free prolongation of Sec. 4.
 *  V [nv x 3] vertices and F [nt x 3] outward triangles of a closed mesh
 *  (host, caller-owned, read during the call); N background resolution
 *  (a power of two); k in {1, 2}; levels L; dirichlet_top nonzero puts
 *  p = 0 on z = 1 (else pure Neumann); coarse_max the dense coarse-solver
 *  limit.  Errors: INVALID (sizes, k, N), OOM. */
typedef struct fvem_grid fvem_grid;

fvem_status fvem_grid_build(const double *V, int64_t nv, const int32_t *F, int64_t nt, int32_t N, int32_t k,
                            int32_t levels, int32_t dirichlet_top, int64_t coarse_max, fvem_grid **out);

/* fvem_grid_build with flags: FVEM_GRID_NAIVE_PROLONGATION builds the naive
 * VEM prolongation of Sec. 4 (shared DOFs copy, every other fine DOF takes
 * the DOF functional of the coarse cell projection, averaged over the coarse
 * cells holding it) instead of the diffusion-free one; its rows reach DOFs
 * of neighbouring coarse cells, so a hierarchy built from it needs the
 * galerkin_general option.  For the ablation of Sec. 4. */
#define FVEM_GRID_NAIVE_PROLONGATION 0x1
fvem_status fvem_grid_build_ex(const double *V, int64_t nv, const int32_t *F, int64_t nt, int32_t N, int32_t k,
                               int32_t levels, int32_t dirichlet_top, int64_t coarse_max, int32_t flags,
                               fvem_grid **out);

/* Fills *d with pointers into the grid's own storage (valid until
 * fvem_grid_destroy); the result can be passed to fvem_hierarchy_build. */
fvem_status fvem_grid_describe(fvem_grid *g, fvem_grid_desc *d);

/* Host views of the finest level: velocity vertices [n_vert x 3], DOF support
 * points [n_dof x 3] and DOF kinds (0 vertex, 1 edge midpoint, 2 face, 3 cell),
 * number of cut trees and of distinct shared element blocks. */
fvem_status fvem_grid_info(fvem_grid *g, const double **vertices, int64_t *n_vert, const double **dof_points,
                           const int8_t **dof_kind, int64_t *n_dof, int64_t *n_trees, int64_t *n_shared);

/* Support points [n_dof x 3] and kinds of level l's free DOFs (vertex, edge
 * midpoint, face vertex mean, cell centroid), in the level's numbering. */
fvem_status fvem_grid_level_points(fvem_grid *g, int32_t level, const double **dof_points, const int8_t **dof_kind,
                                   int64_t *n_dof);

/* Faces of finest-level cell `cell` as outward vertex cycles (velocity
 * vertex ids, counter-clockwise seen from outside), the cell's convex
 * boundary after the conforming overlay (Sec. 5.1).  With face_len and
 * face_vert NULL only the counts are returned; otherwise face_len [cap_faces]
 * receives each face's corner count and face_vert [cap_corners] the corners,
 * face after face (INVALID when a capacity is too small). */
fvem_status fvem_grid_cell_faces(fvem_grid *g, int64_t cell, int32_t *n_faces, int32_t *n_corners,
                                 int32_t *face_len, int32_t *face_vert, int32_t cap_faces, int32_t cap_corners);

void fvem_grid_destroy(fvem_grid *g);

/* ---------------------------------------------------------------- transport
 * The steps on either side of the solve in the simulation loop (Algorithm 1):
 * P2G (Sec. 3.2), the buoyancy force (Sec. 3.2), G2P (Sec. 3.3) and particle
 * advection (Sec. 3.3), on the finest level of a native grid.  A transport
 * copies the grid's BSP trees, boundary triangles and cell geometry to the
 * current device; the grid may be destroyed afterwards.  Positions are
 * [n x 3] FP64 device arrays on the unit cube; cell fields are the
 * projected velocities of fvem_project_velocity (12 per level-0 cell: three
 * components on [1, (x - x_E)/h_E]); vertex fields follow the grid's velocity
 * vertices.  Calls enqueue on hip_stream; fvem_p2g and fvem_advect on one
 * transport must not overlap (else BUSY).  Errors: INVALID, HIP, OOM. */
typedef struct fvem_transport fvem_transport;

fvem_status fvem_transport_create(const fvem_grid *g, void *hip_stream, fvem_transport **out);
void fvem_transport_destroy(fvem_transport *t);

/* Level-0 cell holding each point (the background cell's cube, or the leaf
 * of its BSP tree, Sec. 5.1), -1 in a solid part or outside the unit cube.
 * cell_dev: [n] int32. */
fvem_status fvem_locate(fvem_transport *t, int64_t n, const double *x_dev, int32_t *cell_dev, void *hip_stream);

/* P2G (Sec. 3.2): out[i, :] = sum_p f[p, :] w_ip / sum_p w_ip with
 * w_ip = max(0, 1 - |x_p - x_i|^2 / h^2)^3 over the particles, for every
 * velocity vertex i; 0 where no particle is within h.  f_dev: [n x m]
 * row-major, 1 <= m <= 8; out_dev: [n_vert x m].  Sums run in a fixed order
 * (bitwise reproducible).  Scratch of n entries is kept and grows with n. */
fvem_status fvem_p2g(fvem_transport *t, int64_t n, const double *x_dev, const double *f_dev, int32_t m,
                     double *out_dev, void *hip_stream);

/* The force step of Sec. 3.2 at the vertices: from the P2G fields
 * f [n_vert x m] (columns u_x, u_y, u_z, density, temperature, ...) writes
 * u' [3 n_vert] = u + dt (-alpha density + beta temperature) e_z
 * (Boussinesq buoyancy, +z up). */
fvem_status fvem_buoyancy(fvem_transport *t, const double *f_dev, int32_t m, double alpha, double beta, double dt,
                          double *u_dev, void *hip_stream);

/* G2P (Sec. 3.3): for every particle with ghost[p] == 0 that lies in a fluid
 * cell E, with du = s_new_E(x_p) - s_old_E(x_p),
 * u_p <- a (u_p + du) + (1 - a) s_new_E(x_p) (the FLIP/PIC blend, a in
 * [0, 1]).  s_old is the projection of the P2G velocity before the force. */
fvem_status fvem_g2p(fvem_transport *t, int64_t n, const double *x_dev, const uint8_t *ghost_dev, double *u_dev,
                     const double *s_new_dev, const double *s_old_dev, double a_flip, void *hip_stream);

/* Advection (Sec. 3.3): moves every non-ghost particle that lies in the fluid
 * by midpoint RK2 through the cell field s over dt, in
 * max(1, ceil(dt v N)) substeps (CFL number 1; v the largest |s(x_p)|); a
 * stage that ends outside the fluid is mirrored in the plane of the first
 * boundary triangle or box wall it crosses (up to 4 times), else ends where
 * it began.  *substeps returns the count; more than max_substeps is INVALID.
 * Waits for the speed reduction (one host synchronisation). */
fvem_status fvem_advect(fvem_transport *t, int64_t n, double *x_dev, const uint8_t *ghost_dev, const double *s_dev,
                        double dt, int32_t max_substeps, int32_t *substeps, void *hip_stream);

const char *fvem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FVEM_H */
