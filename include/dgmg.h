/*
 * dgmg.h -- C ABI of the MI355X agglomerated-multigrid PCG solver for the
 * SIPDG-discretised monodomain equations (arXiv 2602.16312).
 *
 * The library solves, at every semi-implicit time step,
 *     (3 chi C_m / (2 dt) M + A) U_{n+1} = I_app - chi M g + chi C_m/(2 dt) M (4 U_n - U_{n-1})
 * (section 3.1, eq. fully_discrete, with ionic current interpolation) by PCG
 * preconditioned with one V-cycle over a nested hierarchy of agglomerated
 * polytopic levels (sections 4 and 5.1; section 6 for the smoother and the
 * V-cycle settings).  All per-step work runs in hand-written gfx950 HIP
 * kernels; setup (assembly, agglomeration, Galerkin products, eigenvalue
 * estimates, coarse factorisation) runs in host C++.
 *
 * Conventions for every entry point:
 *  - Return value: DGMG_OK (0), DGMG_NOT_CONVERGED (+1, outputs and stats
 *    valid) or a negative error code; dgmg_last_error() then returns a
 *    thread-local message.  No C++ exception crosses this boundary.
 *  - "host" pointers are read during the call only; the library copies what
 *    it keeps.  "device" pointers are HIP device memory owned by the caller
 *    (e.g. torch tensors), contiguous, float64, and must stay valid until the
 *    work enqueued on `stream` has completed.
 *  - DG vectors are cell-major: DoF (K, i) lives at K*b + i, b = (p+1)^d, with
 *    the local index i = i0 + (p+1) i1 + (p+1)^2 i2 of the tensor Lagrange
 *    basis on Gauss-Lobatto nodes (x fastest).
 *  - Opaque handles are owned by the library and freed with dgmg_destroy_*.
 *    A solver is not thread-safe; calls that share a solver must be
 *    serialised by the caller.
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *    it; dgmg_pcg_solve and dgmg_time_step synchronise it once per PCG
 *    iteration to read the residual norm for the stopping test.
 */
#ifndef DGMG_H
#define DGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGMG_OK 0
#define DGMG_NOT_CONVERGED 1
#define DGMG_EINVAL (-1)
#define DGMG_ENOTSPD (-2)
#define DGMG_ENAN (-3)
#define DGMG_EHIP (-4)
#define DGMG_ENOMEM (-5)
#define DGMG_EUNSUPPORTED (-6)

#define DGMG_MAX_LEVELS 8

typedef struct dgmg_hierarchy dgmg_hierarchy;
typedef struct dgmg_solver dgmg_solver;

/* Quadrilateral (dim 2) or hexahedral (dim 3) mesh (section 3: shape-regular
 * quad/hex triangulation).  host xyz: n_vert x dim row-major.  host
 * cell_vtx: n_cells x 2^dim vertex ids, corner c = c0 + 2 c1 + 4 c2 at
 * reference point (c0, c1, c2).  Face neighbours must share their face with
 * identical tangential orientation (checked; DGMG_EUNSUPPORTED otherwise). */
typedef struct {
    int32_t dim;
    int64_t n_vert;
    const double* xyz;
    int64_t n_cells;
    const int64_t* cell_vtx;
} dgmg_mesh;

enum { DGMG_AGGLO_GRID = 0, DGMG_AGGLO_RTREE_STR = 1, DGMG_AGGLO_USER = 2 };

/* Agglomeration options (section 4).  n_levels counts the fine mesh too.
 *  GRID:       level l >= 1 groups the fine cells whose centroids (vertex
 *              averages) fall in the same bin of a grid_bins[l][0..dim-1]
 *              grid over the mesh bounding box; bins must nest across levels.
 *  RTREE_STR:  bulk-loaded (sort-tile-recursive) R-tree of fanout
 *              rtree_fanout over the cells' bounding boxes; level l gathers the
 *              leaves below each tree node l levels above the leaves
 *              (Algorithms 1 and 2).
 *  USER:       host user_parents[l-1][e] = level-l id of level-(l-1) entity e. */
typedef struct {
    int32_t n_levels;
    int32_t method;
    int32_t grid_bins[DGMG_MAX_LEVELS][3];
    int32_t rtree_fanout;
    const int64_t* const* user_parents;
} dgmg_agglo_opts;

/* Builds the nested agglomerated hierarchy {T_l} (host only, no device work).
 * The caller's cell numbering is kept: no depth-first permutation of the
 * R-tree's leaves is returned or applied, and vectors stay in the caller's
 * order.  Agglomerates are described by parent arrays
 * (dgmg_hierarchy_parents), which need no contiguity.  The fine level's
 * device layout reads each lower face block transposed from the lower
 * neighbour and coalesces those reads when consecutive cells have
 * consecutive lower neighbours, which a grid (voxel) numbering gives and a
 * tree or space-filling-curve order breaks (a Morton order measured 12%
 * slower on the 1.0M-hex shell).
 * Errors: DGMG_EINVAL for bad sizes, empty agglomerates or a non-nested
 * partition; DGMG_ENOMEM. */
int dgmg_build_hierarchy(const dgmg_mesh* mesh, const dgmg_agglo_opts* opts,
                         dgmg_hierarchy** out);
/* Number of levels, and the number of entities on `level`. */
int dgmg_hierarchy_info(const dgmg_hierarchy* h, int32_t level, int32_t* n_levels,
                        int64_t* n_entities);
/* host out: n_entities(level) parent ids on level+1. */
int dgmg_hierarchy_parents(const dgmg_hierarchy* h, int32_t level, int64_t* out);
/* Bounding boxes of the entities of `level` (level 0: the cells), the
 * boxes that carry the coarse tensor bases (section 5.1): host lo, hi:
 * n_entities(level) x dim, the smallest and largest vertex coordinates of the
 * fine cells an entity contains.  Errors: DGMG_EINVAL (null, level out of
 * range). */
int dgmg_hierarchy_boxes(const dgmg_hierarchy* h, int32_t level, double* lo, double* hi);
void dgmg_destroy_hierarchy(dgmg_hierarchy* h);

enum { DGMG_PENALTY_PAPER = 0, DGMG_PENALTY_FIXED = 1 };
/* Discretisation (section 3): tensor Q_p, 1 <= p <= 4 in 2D, 1 <= p <= 3 in
 * 3D.  Penalty on an
 * interior face: sigma = eta_F * mean(n^T D+ n, n^T D- n) with
 * eta_F = c p(p+1) mean(|F|/|K+|, |F|/|K-|) (PAPER; c = `eta` if > 0, else
 * the paper's c = 1) or eta_F = `eta` (FIXED). */
typedef struct {
    int32_t p;
    int32_t penalty_mode;
    double eta;
} dgmg_disc;

enum { DGMG_MODEL_FHN = 0, DGMG_MODEL_AP = 1, DGMG_MODEL_BO = 2 };
/* Physics (section 2): chi_m, C_m, time step, BDF order (2, or 1 for
 * backward Euler), host D_cell: n_cells x d(d+1)/2 packed symmetric
 * conductivity (xx,xy,yy | xx,xy,xz,yy,yz,zz), host cell_scale: n_cells
 * multipliers of D_K or NULL, ionic model id and its parameter vector
 * (FHN [k,a,eps,Gamma]; AP [k,a,eps0]; BO 28 values in the order documented
 * with the Python binding). */
typedef struct {
    double chi, Cm, dt;
    int32_t bdf;
    const double* D_cell;
    const double* cell_scale;
    int32_t model;
    int32_t n_params;
    const double* params;
} dgmg_physics;

/* Device memory provider for the solver's own buffers (operators, transfer
 * blocks, work vectors and set-up temporaries; e.g. a framework's caching
 * allocator).  alloc returns device memory of at least `bytes` bytes, 256-byte
 * aligned, on the current device, or NULL on failure (the call then fails with
 * DGMG_ENOMEM); free releases a pointer that alloc returned.  alloc is called
 * only inside dgmg_setup_levels, free inside dgmg_setup_levels (set-up
 * temporaries, or everything on an error) and dgmg_destroy_solver; never on
 * the solve or time-stepping path.  ctx is passed through; the functions and
 * ctx must stay valid until dgmg_destroy_solver has returned. */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes);
    void (*free)(void* ctx, void* ptr);
    void* ctx;
} dgmg_allocator;

enum { DGMG_PREC_FP64 = 0, DGMG_PREC_MIXED = 1 };
/* Multigrid options (section 6): Chebyshev-Jacobi degree and number of
 * pre/post sweeps, Lanczos steps, lambda_hi = lam_safety * theta_max,
 * lambda_lo = lambda_hi / smooth_range; host lam_override (NULL or 2 values
 * (lo, hi) per smoothed level) replaces the estimate.  precision MIXED runs
 * the V-cycle in FP32 and the outer PCG in FP64; its coarse inverse is
 * computed in FP64 and kept rounded to FP32 (the coarse GEMV sums in FP64).
 * device_setup = 0 stops after the host setup (inspection on machines
 * without a GPU; solve calls then fail with DGMG_EINVAL).  adjoint = 1 also
 * stores the conductivity derivatives dA/ds_K (cell stiffness and per-side
 * face matrices, FP64) needed by dgmg_grad_accumulate (FHN and AP models).
 * max_rhs (0 or 1: single right-hand side; DGMG_MULTI_RHS: also size every
 * work vector for that many columns, enabling the *_multi calls).  mfma = 1
 * runs the FP32 Chebyshev step of 8-column solves with 8x8 blocks (3D Q1)
 * on the matrix cores (v_mfma_f32_4x4x1f32); 0 keeps it on the vector ALUs.
 * fine_layout selects the device storage of the fine operator: AXIS_ELL
 * stores every face block once (per cell: its block and the blocks of its
 * upper faces along each axis; lower faces are read transposed from the
 * neighbour), TILE_ELL stores each face block twice, oriented for both
 * cells, as on the agglomerated levels; AUTO takes MATRIX_FREE for p >= 2 on
 * meshes of identical boxes with max_rhs <= 1, AXIS_ELL otherwise.  With
 * max_rhs <= 1, AXIS_ELL stores nodal face blocks in sparse form (see
 * dgmg_solver_info.sparse_faces); AXIS_ELL_DENSE keeps every face block
 * whole.
 * MATRIX_FREE (meshes of identical
 * axis-aligned boxes only, single-column calls only; DGMG_EUNSUPPORTED
 * otherwise) stores no fine-level operator: the cell, face and mass terms
 * are evaluated by sum factorisation from the per-cell conductivity.
 * setup_on_device = 1 (needs device_setup = 1) computes the fine operator
 * and mass blocks (except with adjoint = 1), the prolongation blocks, the
 * Galerkin products A_{l+1} = P^T A_l P and the Lanczos estimates on the
 * GPU (the host supplies their integer structure; the blocks are copied
 * back for packing and inspection); 0 computes them on the host.  Both sum
 * in the same order per block.  jacobi selects the Jacobi matrix D of the
 * Chebyshev smoother: POINT the diagonal of A_l (section 6); CELL_BLOCK the
 * cells' b x b diagonal blocks, each inverted once at set-up (host Cholesky;
 * DGMG_ENOTSPD if a block is not positive definite), with the Lanczos
 * estimate taken on L^-1 A_l L^-T, D_K = L_K L_K^T (single-column solvers
 * only: DGMG_EUNSUPPORTED with max_rhs > 1). */
typedef struct {
    int32_t cheb_degree;
    int32_t cheb_sweeps;
    int32_t lanczos_steps;
    double lam_safety;
    double smooth_range;
    const double* lam_override;
    int32_t precision;
    int32_t device_setup;
    int32_t adjoint;
    int32_t max_rhs;
    int32_t mfma;
    int32_t fine_layout;
    int32_t setup_on_device;
    const dgmg_allocator* allocator;  /* NULL: hipMalloc / hipFree; copied at set-up */
    int32_t jacobi;                   /* DGMG_JACOBI_* */
} dgmg_mg_opts;

enum { DGMG_JACOBI_POINT = 0, DGMG_JACOBI_CELL_BLOCK = 1 };

enum { DGMG_LAYOUT_AUTO = 0, DGMG_LAYOUT_TILE_ELL = 1, DGMG_LAYOUT_AXIS_ELL = 2,
       DGMG_LAYOUT_MATRIX_FREE = 3, DGMG_LAYOUT_AXIS_ELL_DENSE = 4 };

/* Number of columns of the multi-right-hand-side calls. */
enum { DGMG_MULTI_RHS = 8 };

/* Assembles A_0 = 3 chi C_m/(2 dt) M + A (eq. fully_discrete; bdf = 1 uses
 * chi C_m/dt), the prolongations, the Galerkin operators A_{l+1} = P^T A_l P
 * (eq. inherited_matrices, Algorithm 3), the smoother data and the dense
 * Cholesky factor of the coarsest operator, and uploads them.  Set-up takes
 * no stream and no separate allocator argument: it mixes host phases with
 * blocking copies and device kernels on the current device's null stream,
 * synchronises the device before returning, and takes the device allocator
 * (if any) from mg->allocator, which it copies.  Errors:
 * DGMG_EINVAL (non-positive Jacobian, bad options), DGMG_ENOTSPD (coarse
 * pivot <= 0), DGMG_EUNSUPPORTED (dim, p), DGMG_EHIP, DGMG_ENOMEM. */
int dgmg_setup_levels(const dgmg_hierarchy* h, const dgmg_disc* disc,
                      const dgmg_physics* phys, const dgmg_mg_opts* mg,
                      dgmg_solver** out);
void dgmg_destroy_solver(dgmg_solver* s);

/* Solver description.  host out arrays sized DGMG_MAX_LEVELS. */
typedef struct {
    int32_t dim, p, b, n_levels, precision, model, n_gates;
    int64_t n_dofs;
    int64_t n_cells[DGMG_MAX_LEVELS];
    int64_t n_faces[DGMG_MAX_LEVELS];
    double lam_lo[DGMG_MAX_LEVELS], lam_hi[DGMG_MAX_LEVELS];
    double op_complexity;
    double t_assembly, t_hierarchy, t_transfer, t_galerkin, t_smoother, t_coarse, t_upload;
    int64_t device_bytes;
    int32_t fine_layout;   /* DGMG_LAYOUT_TILE_ELL, _AXIS_ELL or _MATRIX_FREE as used */
    /* storage of every level's operator as used (0 for the coarsest level,
     * which is solved with its dense inverse); agglomerated levels whose
     * agglomerates form a conforming grid of boxes use AXIS_ELL unless
     * fine_layout = TILE_ELL was asked for */
    int32_t level_layout[DGMG_MAX_LEVELS];
    /* prolongation from level+1 to level: k > 0 when its blocks take only k
     * distinct values (nested boxes) and are stored as a table of those with
     * a type per entity; 0 when every entity's block is stored */
    int32_t prolong_types[DGMG_MAX_LEVELS];
    /* tile-ELL levels: 1 when the cells are assigned to tiles by descending
     * neighbour count within runs of tiles (a tile-to-cell map, kept when it
     * saves at least 3% of the padded slots), 0 for the identity order */
    int32_t level_grouped[DGMG_MAX_LEVELS];
    /* 1 when the fine level's axis-ELL face blocks are stored in sparse form:
     * on a nodal fine level (Lagrange basis on Gauss-Lobatto nodes) entry
     * (i, j) of a face block vanishes unless node i or node j lies on the
     * face (section 3, face terms of a_h), and only the rest is stored.
     * Single-column solvers use it whenever every fine face block has that
     * pattern, unless fine_layout = AXIS_ELL_DENSE was asked for. */
    int32_t sparse_faces;
} dgmg_solver_info;
int dgmg_get_info(const dgmg_solver* s, dgmg_solver_info* info);

enum { DGMG_TOL_REL_R0 = 0, DGMG_TOL_REL_B = 1, DGMG_TOL_ABS = 2 };
typedef struct {
    double tol;
    int32_t tol_mode;
    int32_t max_it;
    int32_t flexible; /* 1: beta = (r_new, z_new - z_old)/(r_old, z_old) */
} dgmg_pcg_opts;
typedef struct {
    int32_t its;      /* A_0 applications inside the loop */
    int32_t converged;
    double r0, rfin;  /* ||b - A x||_2 at start and end */
} dgmg_pcg_stats;

/* PCG on A_0 x = b with one V-cycle per iteration (section 6; section 3.1).
 * device b (N), device x (N; in: initial guess, out: solution).  One
 * right-hand side: several columns go through dgmg_pcg_solve_multi, whose
 * kernels are compiled for a fixed column count (DGMG_MULTI_RHS) and whose
 * stats are per column.  Stops when
 * ||r_k|| <= tol * ||r_0|| (REL_R0), tol * ||b|| (REL_B) or tol (ABS).
 * Errors: DGMG_ENOTSPD on (p, A p) <= 0 or (r, z) <= 0, DGMG_ENAN on a
 * non-finite residual, DGMG_NOT_CONVERGED after max_it. */
int dgmg_pcg_solve(dgmg_solver* s, const double* b, double* x,
                   const dgmg_pcg_opts* opts, dgmg_pcg_stats* stats, void* stream);

/* dgmg_pcg_solve for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same solve, bit-identical results, with the
 * reduction scratch (block partials and the 8 CG scalar slots) in a static
 * per-GPU device array of 1 MiB instead of the solver's buffers.  It calls
 * no hipMalloc, hipFree or allocating library routine; the solver's set-up
 * resolved the array's device address.  Every call on one GPU shares that
 * array and its contents persist between calls (the scalar slots are
 * cleared by a fill kernel on `stream` at entry), so calls that overlap on
 * one GPU, from any solver or stream, race and must be serialised by the
 * caller.  Limit: the solve needs 48 + max(ceil(N / 256), level-0
 * workgroups) doubles of the array's 131,072 (N up to about 31M DoFs);
 * larger solvers get DGMG_EINVAL and must use dgmg_pcg_solve.  Other
 * errors as for dgmg_pcg_solve. */
int dgmg_pcg_solve_noalloc(dgmg_solver* s, const double* b, double* x,
                           const dgmg_pcg_opts* opts, dgmg_pcg_stats* stats, void* stream);

/* Ionic update at every DoF (section 3.1; models of section 2.2).  Takes the
 * four state arrays as separate pointers rather than a dgmg_state, so that the
 * caller chooses where W_{n+1} goes (it may overwrite W_{n-1}, as
 * dgmg_time_step does).  With
 * U* = 2 U - Uprev (BDF2) or U (bdf 1), writes the BDF2 gate update
 * Wnext = (4 W - Wprev + 2 dt c0(U*)) / (3 - 2 dt c1(U*)) for dw/dt = c1 w + c0
 * and g = I_ion(U*, Wnext).  device U, Uprev, g: N; W, Wprev, Wnext: S x N
 * (gate-major).  Wnext may alias Wprev. */
int dgmg_ionic_step(dgmg_solver* s, const double* U, const double* Uprev,
                    const double* W, const double* Wprev, double* Wnext,
                    double* g, void* stream);

/* Caller-owned state of the two-step scheme (device buffers). */
typedef struct {
    double* U;      /* U_n,     N     */
    double* Uprev;  /* U_{n-1}, N     */
    double* W;      /* W_n,     S x N */
    double* Wprev;  /* W_{n-1}, S x N */
    double* g;      /* workspace, N   */
} dgmg_state;

/* One time step t_n -> t_next (section 3.1): ionic update, load vector
 * M f with f = chi C_m/(2 dt)(4 U_n - U_{n-1}) + I_app - chi g (ICI), PCG
 * warm-started from U_n.  device iapp: N nodal applied current or NULL,
 * already evaluated at t_next by the caller; t_next itself is not read (the
 * scheme's coefficients do not depend on t, and the caller owns the clock).  On
 * return the pointer pairs of *state are rotated: U holds U_{n+1}, Uprev
 * U_n, W holds W_{n+1}, Wprev W_n (no data is copied).  Errors as for
 * dgmg_pcg_solve. */
int dgmg_time_step(dgmg_solver* s, dgmg_state* state, double t_next,
                   const double* iapp, const dgmg_pcg_opts* opts,
                   dgmg_pcg_stats* stats, void* stream);

/* Multi-right-hand-side PCG: nrhs (= DGMG_MULTI_RHS) independent systems
 * A_0 x_c = b_c sharing one operator and one V-cycle per iteration, each
 * column with its own CG scalars alpha_c, beta_c and its own stopping test
 * (a converged column is frozen while the others iterate).  device b, x:
 * N x nrhs, column-minor (entry (DoF t, column c) at t*nrhs + c).  host stats:
 * nrhs entries.  Requires max_rhs >= nrhs at set-up.  Returns DGMG_OK when
 * every column converged, DGMG_NOT_CONVERGED otherwise; errors as for
 * dgmg_pcg_solve (on any active column). */
int dgmg_pcg_solve_multi(dgmg_solver* s, int32_t nrhs, const double* b, double* x,
                         const dgmg_pcg_opts* opts, dgmg_pcg_stats* stats, void* stream);

/* dgmg_time_step for nrhs independent simulations sharing the mesh, the
 * conductivity and the solver (e.g. different stimulus sites): every state
 * buffer and iapp hold nrhs columns, column-minor (U: N x nrhs, W: S x N x
 * nrhs), stats nrhs entries. */
int dgmg_time_step_multi(dgmg_solver* s, int32_t nrhs, dgmg_state* state, double t_next,
                         const double* iapp, const dgmg_pcg_opts* opts,
                         dgmg_pcg_stats* stats, void* stream);

/* ---- operator-level entry points (parity tests, adjoint driver) ---- */

/* y = A_level x.  prec selects the stored FP64 or FP32 copy of the level
 * (FP32 exists for every level in MIXED mode); device x, y: N_level float64. */
int dgmg_apply(dgmg_solver* s, int32_t level, int32_t prec, const double* x,
               double* y, void* stream);
/* z = B r, one V-cycle in the solver's precision mode; device r, z: N. */
int dgmg_vcycle(dgmg_solver* s, const double* r, double* z, void* stream);
/* dgmg_apply and dgmg_vcycle on nrhs (= DGMG_MULTI_RHS) column-minor
 * columns (N_level x nrhs); the V-cycle is applied to every column. */
int dgmg_apply_multi(dgmg_solver* s, int32_t level, int32_t prec, int32_t nrhs,
                     const double* x, double* y, void* stream);
int dgmg_vcycle_multi(dgmg_solver* s, int32_t nrhs, const double* r, double* z,
                      void* stream);
/* b = M f per cell (the ICI load vector); device f, b: N. */
int dgmg_mass_apply(dgmg_solver* s, const double* f, double* b, void* stream);

/* Host copies of a level's FP64 operator: diag (n_cells x b x b, row-major
 * blocks), faces as (plus, minus) cell pairs and blocks A(plus rows, minus
 * cols), prolongation blocks to this level from level+1 (n_cells x b x b) and
 * parents.  Any out pointer may be NULL; sizes from dgmg_get_info. */
int dgmg_export_level(const dgmg_solver* s, int32_t level, double* diag,
                      int64_t* face_cells, double* face_blocks, double* prolong,
                      int64_t* parents);

/* ---- discrete adjoint (gradient of a sensor misfit with respect to the
 * per-cell conductivity scalings s_K, D_K -> s_K D_K; extension of the
 * time stepping of section 3.1).  A(s) = sum_K s_K dA/ds_K. ---- */

/* Sensors: host cells (n) and host reference points (n x dim, in [0,1]^dim)
 * of the evaluation functionals e_k^T U = sum_i U[cell_k, i] phi_i(ref_k). */
int dgmg_set_sensors(dgmg_solver* s, int32_t n, const int64_t* cells, const double* ref);
/* r_k = e_k^T U - target_k (device target: n floats); device loss[0] +=
 * sum_k r_k^2; when device Ubar (N) is non-NULL, Ubar += sum_k 2 r_k e_k. */
int dgmg_sensor_misfit(dgmg_solver* s, const double* U, const double* target, double* Ubar,
                       double* loss, void* stream);
/* Reverse of the ionic update and load vector of the step that produced
 * U_{n+1} from the state (U = U_n, Uprev = U_{n-1}, W = W_n, Wprev = W_{n-1}):
 * given device lambda = A_0^-1 Ubar_{n+1} (N) and the incoming adjoint of
 * W_{n+1} (device Wbar_in, S x N), accumulates into device Ubar (of U_n),
 * Uprevbar (of U_{n-1}), Wbar (of W_n), Wprevbar (of W_{n-1}).  Needs
 * adjoint = 1 at set-up. */
int dgmg_adjoint_step(dgmg_solver* s, const double* U, const double* Uprev, const double* W,
                      const double* Wprev, const double* lambda, const double* Wbar_in, double* Ubar,
                      double* Uprevbar, double* Wbar, double* Wprevbar, void* stream);
/* device grad[K] += -lambda^T (dA/ds_K) U over the cell and face blocks of K
 * (device lambda, U: N; grad: n_cells).  Needs adjoint = 1 at set-up. */
int dgmg_grad_accumulate(dgmg_solver* s, const double* lambda, const double* U, double* grad,
                         void* stream);

/* Kernel timing with HIP events recorded on the caller's stream around every
 * launch of one kernel kind on one level, between begin and end: kind 0 the
 * fused Chebyshev step, 1 the fused residual, 2 the plain/dot apply, 3 the
 * restriction (level = fine level), 4 the prolongation (level = fine level),
 * 5 the coarse solve (level ignored).  end waits for the recorded events and
 * returns the number of launches and their summed duration in ms. */
int dgmg_profile_begin(dgmg_solver* s, int32_t kind, int32_t level);
int dgmg_profile_end(dgmg_solver* s, int64_t* launches, double* total_ms);

/* Per-phase times of the time step (the semi-implicit step of section 3.1:
 * ionic update, load vector, PCG solve), for per-step logs.  With on = 1
 * every following dgmg_time_step records HIP events on its stream at the
 * phase boundaries (extra event packets: leave it off in timed runs);
 * on = 0 stops that.  dgmg_step_phase_ms waits for the last such step's
 * final event and writes its three durations in ms to ms[0] (ionic update),
 * ms[1] (load vector) and ms[2] (PCG solve, host stopping tests included).
 * Errors: DGMG_EINVAL for a null argument, or from dgmg_step_phase_ms when
 * no step was timed since phase timing was switched on. */
int dgmg_set_phase_timing(dgmg_solver* s, int32_t on);
int dgmg_step_phase_ms(dgmg_solver* s, double* ms);

/* Average duration (ms, HIP events on `stream`) of `reps` back-to-back
 * launches of one smoother kernel (kind 0: fused Chebyshev step, 1: fused
 * residual) on `level` < n_levels - 1, in the solver's V-cycle precision,
 * on nrhs (1 or DGMG_MULTI_RHS) columns.  Uses the level's internal work
 * vectors only (their contents are overwritten); caller data are untouched. */
int dgmg_kernel_bench(dgmg_solver* s, int32_t kind, int32_t level, int32_t nrhs, int32_t reps,
                      void* stream, double* avg_ms);

const char* dgmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DGMG_H */
