/*
 * cbs.h -- C ABI of the MI355X coupled block-sparse solver (libcbs.so).
 *
 * The library solves the assembled coupled system of arXiv 2403.07882,
 * Eq. (coupl_system):  A_ii U_i + sum_N A_ij U_j = b_i,  with dense n x n
 * blocks (n = 4 for the pressure-based p-U system of Sec. 2.2, n = 5 for the
 * density-based system of Sec. 2.1) on a face-neighbour stencil, by an
 * aggregation-AMG-preconditioned Krylov method (BiCGStab or flexible GMRES,
 * the solver families of Sec. 2.3).  The call sequence follows the lifecycle
 * of Algorithm amgxFoam: create from the face-addressed LDU form (pattern set
 * up once per topology), replace values when only coefficients change,
 * set up the preconditioner, solve (with the caller's x as initial guess),
 * read statistics, destroy.
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer (e.g. a torch tensor's
 *    data_ptr()) unless the comment says "host".  The library never takes
 *    ownership of caller arrays: they are borrowed for the duration of the
 *    call (and of the work it enqueues on the handle's stream).
 *  - Blocks are n x n, row-major, packed one after another (Sec. 2.3, Fig.
 *    block_amgx).  Vectors are block AoS: x[i*n + v] is variable v of cell i.
 *  - LDU reading (the paper names only "OpenFOAM native LDU storage"):
 *    upper[f] is the block at (row lower_addr[f], column upper_addr[f]) and
 *    lower[f] the block at (row upper_addr[f], column lower_addr[f]).  Faces
 *    may come in any order and with either orientation.
 *  - All work is enqueued on the stream given at creation (a hipStream_t
 *    passed as void*; NULL = the default stream).  Entry points that return
 *    results to the host (statistics, error flags) synchronise that stream.
 *  - Return value: 0 = CBS_OK; > 0 = warning (outputs written); < 0 = error.
 *    cbs_last_error() gives a thread-local message with detail (e.g. the
 *    index of a singular block).  No C++ exception crosses this boundary.
 *  - A handle is not thread-safe: use one host thread per handle.
 */
#ifndef CBS_H
#define CBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cbs_system *cbs_handle;

enum cbs_status {
    CBS_OK = 0,
    CBS_NOT_CONVERGED = 1,   /* iteration cap reached; x and stats still written */
    CBS_ERR_ARG = -1,        /* bad argument (size, NULL pointer, bdim out of 1..5) */
    CBS_ERR_PATTERN = -2,    /* face index out of range, self face, duplicate face */
    CBS_ERR_SINGULAR = -3,   /* a diagonal block (any level) or coarse matrix is singular */
    CBS_ERR_BREAKDOWN = -4,  /* Krylov breakdown persisted after one restart */
    CBS_ERR_NONFINITE = -5,  /* NaN/Inf in matrix values or right-hand side */
    CBS_ERR_STATE = -6,      /* call out of order (e.g. solve before setup) */
    CBS_ERR_OOM = -7,        /* device allocation failed */
    CBS_ERR_HIP = -8         /* HIP runtime error */
};

/* Krylov methods of Sec. 2.3: BiCGStab; flexible GMRES(m), which stores the
 * m preconditioned basis vectors; right-preconditioned GMRES(m), which stores
 * only the basis and applies the preconditioner once more per restart cycle
 * (the same iterates as FGMRES when the preconditioner is a fixed linear
 * operator, with m fewer N*n vectors in device memory). */
enum { CBS_SOLVER_BICGSTAB = 0, CBS_SOLVER_FGMRES = 1, CBS_SOLVER_GMRES = 2 };
/* Preconditioners: none; block Jacobi (D^{-1}); the aggregation-AMG V-cycle;
 * multicolour symmetric block Gauss-Seidel on the whole system, the GMRES +
 * SGS configuration of the CRM runs (Sec. 4.1): max(1, pre_sweeps) symmetric
 * steps from z = 0, FP64 whatever the precision option, the colour classes
 * of a graph colouring of the block pattern in ascending then descending
 * order.  Colours are computed at cbs_setup (CBS_ERR_ARG beyond 128). */
enum { CBS_PREC_NONE = 0, CBS_PREC_BJACOBI = 1, CBS_PREC_AMG = 2, CBS_PREC_SGS = 3 };
/* AMG smoothers (Sec. 2.3): damped block Jacobi; multicolour block DILU;
 * multicolour symmetric block Gauss-Seidel (one step = the colours in order,
 * then in reverse, each row x_i = D_i^{-1} (b_i - sum_{j != i} A_ij x_j));
 * multicolour block ILU(0) (the incomplete-LU smoother: A ~ L U in the
 * colour order, no fill outside A's block pattern; one step
 * x += (L U)^{-1} (b - A x)).  On a block graph without triangles (a hex
 * mesh) ILU(0) and DILU are the same preconditioner.  DILU, Gauss-Seidel and
 * ILU(0) run on the dilu_levels finest levels. */
enum { CBS_SMOOTH_BJACOBI = 0, CBS_SMOOTH_DILU = 1, CBS_SMOOTH_SGS = 2, CBS_SMOOTH_ILU0 = 3 };
enum { CBS_PRECISION_FP64 = 0, CBS_PRECISION_MIXED = 1 };

/* Solver options (the "linear solver options" of Algorithm amgxFoam).
 * cbs_default_options() fills the defaults given in brackets. */
typedef struct cbs_options {
    int32_t solver;          /* CBS_SOLVER_*                         [BICGSTAB] */
    int32_t restart;         /* (F)GMRES restart length m            [30] */
    int32_t precond;         /* CBS_PREC_*                           [AMG] */
    int32_t smoother;        /* CBS_SMOOTH_* (AMG levels)            [BJACOBI] */
    int32_t pre_sweeps;      /* smoothing sweeps before coarse corr. [2] */
    int32_t post_sweeps;     /* smoothing sweeps after coarse corr.  [2] */
    double omega;            /* block-Jacobi damping                 [0.9] */
    double tol;              /* stop at ||b - A x||_2 / ||b||_2 <= tol [1e-8] */
    int32_t max_iter;        /* outer Krylov iteration cap           [500] */
    int32_t precision;       /* CBS_PRECISION_*: MIXED = FP32 hierarchy and
                                smoothers inside the FP64 Krylov loop [FP64] */
    int32_t coarse_max;      /* coarsest level: <= this many block rows per
                                system, solved by a dense FP64 inverse [16] */
    int32_t match_passes;    /* pairwise-matching passes per level   [2] */
    int32_t max_levels;      /* hierarchy depth cap                  [24] */
    int32_t reuse_aggregates;/* cbs_setup again after cbs_update_values: keep
                                the aggregates, redo only the numeric part [0] */
    int32_t check_every;     /* read the convergence flag back every k
                                iterations (device-side early exit)  [1] */
    int32_t renumber;        /* AMG only: renumber rows internally so that
                                every aggregate (at every level) is a
                                contiguous row range, which keeps vector
                                gathers cache-local on irregularly numbered
                                meshes; inputs and outputs keep the caller's
                                numbering                            [1] */
    int32_t dilu_levels;     /* smoother DILU, SGS or ILU0: the dilu_levels finest
                                levels use it, coarser ones damped block
                                Jacobi; < 0 = every level            [2] */
    int32_t row_split;       /* block-row kernels on levels of fewer than
                                32,768 block rows: threads that share one
                                scalar row (1, 2, 4, 8 or 16); 0 = chosen from
                                the level's mean row length. Changes only the
                                order of the row sums                [0] */
    int32_t tail_rows;       /* AMG V-cycle: from the first level of at most
                                this many block rows (all systems together)
                                down to the coarsest and back, the cycle runs
                                in one workgroup (one kernel instead of about
                                five per level); 0 = 256, < 0 = never. Changes
                                only the order of the row sums       [0] */
    int32_t schedule;        /* schedule of the block-row kernels (blocks
                                loaded per step, non-temporal matrix loads):
                                0 = timed on the level-0 operator at setup
                                (levels of >= 65,536 block rows); 1..6 force
                                (unroll, non-temporal) = (1,0), (1,1), (2,0),
                                (2,1), (4,0), (4,1) on every level in both
                                precisions. Changes only the order of
                                the row sums                         [0] */
    int32_t scaled_sweeps;   /* mixed precision, block-Jacobi levels: sweeps
                                on the row-scaled values D_i^{-1} A_ij rounded
                                once to FP32, the FP64 D^{-1} applied only by
                                the zero-guess sweep (1), or every sweep on
                                the FP32 A_ij with the FP64 D^{-1} (0)   [1] */
    int32_t w_levels;        /* AMG cycle shape (Sec. 2.3 names the multigrid
                                cycle, not its shape): on each of the
                                w_levels finest levels the coarse correction
                                runs the next level's cycle twice, the second
                                run starting from the first one's result (a
                                W-cycle on those levels); a level whose next
                                level is the coarsest runs it once, since
                                that level is solved exactly. 0 = V-cycle;
                                beyond the depth: every level (W-cycle).
                                The single-workgroup tail starts below these
                                levels                               [0] */
    double coarse_omega;     /* block-Jacobi damping on every level below the
                                finest; 0 = omega there too (the paper
                                leaves the damping open)             [0] */
} cbs_options;

/* Per-solve statistics (Algorithm amgxFoam: iterations and residuals). */
typedef struct cbs_stats {
    int32_t iterations;
    int32_t status;              /* the cbs_status of this system's solve */
    int32_t levels;              /* AMG levels (1 = no coarsening) */
    int32_t precision_fallback;  /* 1 if a mixed solve escalated to FP64 */
    double rel_res_true;         /* ||b - A x|| / ||b|| recomputed in FP64 at exit */
    double rel_res_recursive;    /* the Krylov recurrence's estimate where the
                                    solver stopped, before the true residual is
                                    recomputed (BiCGStab: the updated r;
                                    (F)GMRES: the least-squares residual of the
                                    last cycle) */
    double rel_res_initial;      /* ||b - A x0|| / ||b|| */
    double t_convert_ms;         /* last LDU -> block-CSR value conversion */
    double t_setup_ms;           /* last cbs_setup */
    double t_solve_ms;           /* this solve */
    double op_complexity;        /* sum_l nnzb_l / nnzb_0 */
} cbs_stats;

void cbs_default_options(cbs_options *opt /* host */);

/* Create a system from the face-addressed LDU form and convert it to block
 * CSR on the device (the permutation step of Algorithm amgxFoam, Sec. 2.3):
 * pattern (row_ptr, ascending columns, diagonal inline) and values, bit-exact.
 *   n_cells  N >= 1 block rows; n_faces F >= 0 internal faces; bdim n in 1..5
 *   lower_addr[F], upper_addr[F]  int32 cell indices, 0 <= . < N, l != u,
 *                                 each unordered pair at most once
 *   diag[N*n*n], upper[F*n*n], lower[F*n*n]   FP64 blocks
 *   stream   hipStream_t as void*; all later work of the handle runs on it
 * Errors: CBS_ERR_ARG, CBS_ERR_PATTERN, CBS_ERR_NONFINITE, CBS_ERR_OOM,
 * CBS_ERR_HIP.  On error *out is NULL and nothing leaks. */
int cbs_create_from_ldu(cbs_handle *out /* host */, int32_t n_cells, int32_t n_faces,
                        int32_t bdim, const int32_t *lower_addr, const int32_t *upper_addr,
                        const double *diag, const double *upper, const double *lower,
                        void *stream);

/* Batched create: n_sys independent systems concatenated (the offset layout
 * of the partition consolidation in Sec. 2.3).  cell_off[n_sys+1] and
 * face_off[n_sys+1] are HOST int64 prefix offsets; the face address arrays
 * hold per-system LOCAL cell indices; the value arrays are concatenated.
 * Every system converges on its own (per-system scalars and masks). */
int cbs_create_batch_from_ldu(cbs_handle *out /* host */, int32_t n_sys,
                              const int64_t *cell_off /* host */, const int64_t *face_off /* host */,
                              int32_t bdim, const int32_t *lower_addr, const int32_t *upper_addr,
                              const double *diag, const double *upper, const double *lower,
                              void *stream);

/* Replace the coefficients, same pattern (the coefficient-replacement step of
 * Algorithm amgxFoam).  Invalidates the preconditioner: call cbs_setup again
 * (reuse_aggregates = 1 keeps the coarsening). */
int cbs_update_values(cbs_handle h, const double *diag, const double *upper, const double *lower);

/* Assemble the density-based coupled matrix on the device, straight into the
 * handle's block-CSR values: V/dtau I - dR/dQ of Eq. (discretBackward) with
 * the approximate Jacobian of Eqs. (approxJac1, approxJac2), Sec. 2.1.  Takes
 * the place of cbs_update_values (same pattern, same follow-up: cbs_setup).
 * Block size 5, unknowns (rho, rho u, rho v, rho w, rho E).
 *   Q[N*5]        conservative state per cell (device)
 *   Sf[F*3]       face area vectors S_f n_f, pointing from lower_addr[f]
 *                 (row of the upper block) to upper_addr[f] (device)
 *   lam_visc[F]   viscous spectral radius per unit area, added to the
 *                 convective radius of the Roe-averaged face state (device;
 *                 NULL = 0)
 *   v_dt[N]       V/dtau per cell, added to the diagonal (device; NULL = 0)
 *   gamma         ratio of specific heats (> 1)
 * Face f with owner l, neighbour u, s = Sf[f], S lambda = |u~.s| + c~|s| +
 * |s| lam_visc[f] (Roe averages, c~^2 = (gamma-1)(H~ - |u~|^2/2)):
 *   A_ll += (J(Q_l, s) + S lambda I)/2,   A_lu = (J(Q_u, s) - S lambda I)/2,
 *   A_uu += (-J(Q_u, s) + S lambda I)/2,  A_ul = (-J(Q_l, s) - S lambda I)/2,
 * J(Q, s) the Euler convective flux Jacobian d(F(Q).s)/dQ of an ideal gas.
 * Interior faces only: boundary contributions belong in v_dt or come from
 * cbs_update_values.  Batched handles take the concatenated cells and faces.
 * Errors: CBS_ERR_ARG (bdim != 5, NULL Q, NULL Sf with faces, gamma <= 1),
 * CBS_ERR_NONFINITE (a cell state with non-positive density or pressure, or
 * a non-finite assembled coefficient). */
int cbs_assemble_luo(cbs_handle h, const double *Q, const double *Sf, const double *lam_visc, const double *v_dt,
                     double gamma);

/* cbs_assemble_luo for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as cbs_assemble_luo; the
 * per-face and per-cell intermediates live in a fixed 64 MiB array that the
 * library holds on every device it runs on until the process ends, instead
 * of buffers of the handle.  No hipMalloc, hipFree or other allocating call
 * is made.  Limit: 8 * (32 + F' + N5' + N4') bytes <= 64 MiB, where F', N5'
 * and N4' are F, 5N and 4N rounded up to multiples of 32 (about 699,000 hex
 * cells); a larger system returns CBS_ERR_ARG before any work.  Every call
 * on one device shares that array: calls that overlap on one GPU (handles on
 * different streams) race and must be serialised by the caller.  The handle
 * must be used with the device current at its creation. */
int cbs_assemble_luo_noalloc(cbs_handle h, const double *Q, const double *Sf, const double *lam_visc,
                             const double *v_dt, double gamma);

/* Assemble the pressure-based coupled matrix on the device, straight into
 * the handle's block-CSR values: the face coefficients of Sec. 2.2 (after
 * Eq. prb_coeff).  Takes the place of cbs_update_values.  Block size 4,
 * unknowns (p, Ux, Uy, Uz); row 0 is continuity.  All arrays on the device.
 *   Sf[F*3]     face area vectors, from lower_addr[f] (owner) to upper_addr[f]
 *   fx[F]       the owner's linear-interpolation weight at the face
 *   d[F*3]      centroid distance x_upper - x_lower
 *   flux[F]     previous-iteration volume flux u_f . Sf out of the owner
 *   nu_eff[F]   laminar + turbulent viscosity at the face
 *   vol[N]      cell volumes
 *   uu_add[N], pp_add[N]  added to the momentum (times I) and pressure
 *               diagonals: boundary faces and relaxation (NULL = 0)
 * Per face, seen from row i (area vector s out of i, flux F_i = u_f . s, own
 * weight w, k = nu_eff |S| / (n . d)): a_ii^uu += (max(F_i, 0) + k) I,
 * a_ij^uu = -(max(-F_i, 0) + k) I; a_ii^up = a_ii^pu += w s,
 * a_ij^up = a_ij^pu = (1 - w) s; with D_i = V_i / a_ii^uu (every face and
 * uu_add summed) and D_f the interpolated D, a_ij^pp = -D_f |S| / (n . d) and
 * a_ii^pp += D_f |S| / (n . d) (the Rhie-Chow Laplacian, positive diagonal).
 * Errors: CBS_ERR_ARG (bdim != 4, NULL arrays), CBS_ERR_NONFINITE (a zero
 * momentum diagonal or n . d = 0). */
int cbs_assemble_pu(cbs_handle h, const double *Sf, const double *fx, const double *d, const double *flux,
                    const double *nu_eff, const double *vol, const double *uu_add, const double *pp_add);

/* Device memory of a handle through the caller's allocator (for example a
 * framework's caching allocator).  The library keeps its own cache of blocks
 * on top of it, keyed by stream and allocator: alloc is called only when no
 * cached block of the handle's stream fits, and free when blocks are given
 * back (at cbs_destroy of the handle).  alloc(ctx, bytes, stream) returns a
 * device pointer aligned to 256 bytes, or NULL (the call that needed it then
 * fails with CBS_ERR_OOM); free(ctx, ptr, stream) releases one.  stream is
 * the handle's stream, the only stream the memory is used on.  Both run on
 * the thread that called into the library. */
typedef struct cbs_allocator {
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
    void *ctx;
} cbs_allocator;

/* Allocations of h from this call on go through *a (NULL: back to hipMalloc
 * / hipFree).  Blocks made earlier stay with the allocator that made them
 * and are given back to it.  *a is copied; its functions and ctx must stay
 * valid until cbs_destroy(h) returns.  Errors: CBS_ERR_ARG (NULL handle, or
 * an allocator with alloc or free missing). */
int cbs_set_allocator(cbs_handle h, const cbs_allocator *a /* host, may be NULL */);

/* Build the preconditioner: block-diagonal inverses (FP64), and for AMG the
 * pairwise-matching aggregation, Galerkin coarse operators P^T A P with
 * piecewise-constant P, FP32 level copies (mixed precision) and the dense
 * FP64 inverse of each coarsest system.  opt may be NULL (defaults).
 * Errors: CBS_ERR_SINGULAR (cbs_last_error names level and block). */
int cbs_setup(cbs_handle h, const cbs_options *opt /* host */);

/* Solve A x = b.  b[N*n] in; x[N*n] is the initial guess on entry (warm
 * start, as Algorithm amgxFoam uploads the current solution) and the
 * solution on exit.  st: host, may be NULL; for a batch, an array of n_sys.
 * b = 0 returns x = 0 with 0 iterations.  Returns CBS_NOT_CONVERGED (x
 * written) at the iteration cap. */
int cbs_solve(cbs_handle h, const double *b, double *x, cbs_stats *st /* host */);

/* The batched solve of a handle from cbs_create_batch_from_ldu: the same
 * call as cbs_solve, spelled for batches.  b and x are the systems'
 * vectors concatenated in system order (x[cell_off[s]*n ..] is system s);
 * st_array (host, may be NULL) receives n_sys stats, one per system, each
 * system stopping at its own tolerance.  Returns CBS_NOT_CONVERGED when any
 * system stops at the iteration cap (every x written). */
int cbs_solve_batch(cbs_handle h, const double *b, double *x, cbs_stats *st_array /* host */);

/* Solve the transposed system A^T lambda = g with the same options and
 * aggregates (the adjoint solve of L(x(A,b))).  Same argument rules as
 * cbs_solve (lambda in = initial guess). */
int cbs_solve_transpose(cbs_handle h, const double *g, double *lambda, cbs_stats *st /* host */);

/* Gradient of a scalar L(x) w.r.t. the LDU values given lambda = A^{-T} dL/dx
 * and the solution x:  grad_diag[i] = -lambda_i x_i^T,
 * grad_upper[f] = -lambda_{l(f)} x_{u(f)}^T, grad_lower[f] = -lambda_{u(f)} x_{l(f)}^T
 * (dL/db = lambda itself).  Outputs are N*n*n and F*n*n FP64 blocks. */
int cbs_gradient(cbs_handle h, const double *lambda, const double *x,
                 double *grad_diag, double *grad_upper, double *grad_lower);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), FP64, block AoS. */
int cbs_spmv(cbs_handle h, const double *x, double *y, int32_t transpose);

/* One application z = M^{-1} r of the preconditioner built by cbs_setup
 * (zero initial guess), in the configured precision. */
int cbs_apply_precond(cbs_handle h, const double *r, double *z);

/* The preconditioner of the transposed solve (reading of Sec. 2.3 for the
 * adjoint: the same aggregates, Galerkin operators of A^T, block-Jacobi or
 * DILU factors of A^T): one application z = M_T^{-1} r, zero initial guess,
 * in the configured precision.  Builds the transposed hierarchy on first use
 * after cbs_setup, as cbs_solve_transpose does. */
int cbs_apply_precond_transpose(cbs_handle h, const double *r, double *z);

/* Kernel-level access to the smoother of one AMG level, for verification and
 * for timing the kernels the V-cycle runs (Sec. 2.3, smoothers).  Works on
 * level `level` (0 .. levels-2; the coarsest level has no smoother) of the
 * hierarchy from the last cbs_setup, in its internal row numbering, on device
 * vectors b, x, y of n_rows(level)*bdim values in the precision the hierarchy
 * runs in, reported in *fp32 when fp32 is not NULL (1: float, mixed precision
 * without escalation; 0: double).  All three vectors NULL: only *fp32 is
 * written.
 *   op CBS_LEVEL_SWEEP:    one damped block-Jacobi sweep from x,
 *                          y = x + omega Dinv (b - A x); in mixed precision the
 *                          sweep runs on the row-scaled values Dinv A, so b
 *                          must already be the scaled right side Dinv b.
 *   op CBS_LEVEL_RESIDUAL: y = b - A x.
 * y must not alias x.  Errors: CBS_ERR_STATE before cbs_setup, without the
 * AMG preconditioner, or for a sweep on a DILU level; CBS_ERR_ARG for a bad
 * level or op or a partial set of NULL vectors. */
enum { CBS_LEVEL_SWEEP = 0, CBS_LEVEL_RESIDUAL = 1 };
int cbs_level_apply(cbs_handle h, int32_t level, int32_t op, const void *b, const void *x, void *y,
                    int32_t *fp32 /* host, may be NULL */);

/* Field packing around the solve (Algorithm amgxFoam, first and last steps):
 * soa[v*N + i] (one array per variable) <-> aos[i*n + v].  Bit-exact. */
int cbs_pack_fields(int32_t n_cells, int32_t bdim, const double *soa, double *aos, void *stream);
int cbs_unpack_fields(int32_t n_cells, int32_t bdim, const double *aos, double *soa, void *stream);

/* Introspection for verification.  Sizes: cbs_get_info fills any non-NULL
 * host scalar.  cbs_get_bcsr copies the level-0 block CSR and the slot maps
 * (diag_slot[N], upper_slot[F], lower_slot[F]) into device arrays of the
 * caller (any pointer may be NULL to skip it). */
int cbs_get_info(cbs_handle h, int32_t *n_cells /* host */, int32_t *n_faces /* host */,
                 int32_t *bdim /* host */, int64_t *nnzb /* host */, int32_t *levels /* host */,
                 int32_t *n_sys /* host */);
int cbs_get_bcsr(cbs_handle h, int32_t *row_ptr, int32_t *col, double *vals,
                 int32_t *diag_slot, int32_t *upper_slot, int32_t *lower_slot);

/* The transpose-slot map of the level-0 block CSR, mirror[nnzb] (device
 * array of the caller): mirror[k] is the slot of block (j, i) for the block
 * (i, j) in slot k.  It is what the transposed product and solve read A^T
 * through (Eq. discretBackward's adjoint): mirror[upper_slot[f]] =
 * lower_slot[f], mirror[lower_slot[f]] = upper_slot[f], and a diagonal slot
 * is its own mirror. */
int cbs_get_mirror(cbs_handle h, int32_t *mirror);

/* Level l of the AMG hierarchy (after cbs_setup): n_rows, nnzb (host) and,
 * into caller device arrays when non-NULL, its block CSR (FP64 values) in
 * the internal row numbering, the aggregate map agg[n_rows] to level l+1
 * (coarsest level: not written), the DILU colour of each row (colour[n_rows],
 * DILU smoother only) and order[n_rows]: the row of the previous numbering
 * that internal row i' holds (level 0: the caller's cell index; identity
 * when renumbering is off). */
int cbs_get_level(cbs_handle h, int32_t level, int32_t *n_rows /* host */, int64_t *nnzb /* host */,
                  int32_t *row_ptr, int32_t *col, double *vals, int32_t *agg, int32_t *colour,
                  int32_t *order);

/* Free every device buffer of the handle (Algorithm amgxFoam, final step).
 * NULL is allowed. */
int cbs_destroy(cbs_handle h);

const char *cbs_error_string(int code);
const char *cbs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CBS_H */
