/*
 * blockoa.h -- C ABI of the MI355X (gfx950) block Krylov + operator action
 * data path for steady IC thermal simulation.
 *
 * The path follows the three steps of the paper's method (Sec. III):
 *   1. basis solutions: one shared-operator block solve A X = B for s power
 *      maps at once (Sec. III-A, Eq. (4));
 *   2. temperature fields T = X C, random combinations of the basis
 *      solutions (Sec. III-B, Eq. (5));
 *   3. operator action F = A T, recovering each field's heat source without
 *      a solve (Sec. III-C, Eq. (6)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are DEVICE pointers unless marked "host".  Matrices are column
 *   major with an explicit leading dimension (element (i, j) at
 *   ptr[i + j * ld]); each column of an N x s or N x M block is one field
 *   over the grid, flattened x-fastest, then y, then z (layer 0 bottom).
 * - The caller owns every buffer (operator coefficients, workspace, inputs,
 *   outputs).  The library never allocates device memory.  Handles own host
 *   metadata only.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Kernels run on that stream.
 * - Every argument is validated before any launch.  Bad arguments return
 *   BKO_EINVAL and launch nothing.  No call aborts the process and no C++
 *   exception crosses the ABI.  The message of the last failure on the
 *   calling thread is returned by bko_last_error().
 * - bko_combine and bko_apply_operator are stream-asynchronous: a BKO_OK
 *   return means the launch was accepted.  bko_assemble_heat_operator and
 *   bko_block_krylov_solve synchronise the stream before returning.
 *
 * Dtype legend: BKO_F64 = IEEE double, BKO_F32 = IEEE single, BKO_BF16 =
 * bfloat16 stored as 16-bit words (round-to-nearest-even on conversion).
 */
#ifndef BLOCKOA_H
#define BLOCKOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BKO_OK = 0,
    BKO_EINVAL = 1,      /* bad argument; nothing launched                     */
    BKO_ENOTSPD = 2,     /* operator not positive definite (e.g. k <= 0)       */
    BKO_ENOCONV = 3,     /* solve hit max_iter; X holds the last iterate       */
    BKO_EBREAKDOWN = 4,  /* every search direction deflated before tol        */
    BKO_EHIP = 5,        /* HIP runtime error (launch / copy / sync)           */
    BKO_ENOMEM = 6,      /* caller buffer smaller than the queried size        */
    BKO_ENOTIMPL = 7
} bko_status;

typedef enum { BKO_F64 = 0, BKO_F32 = 1, BKO_BF16 = 2 } bko_dtype;

/* Boundary face models of Sec. II-A with homogeneous data: the unknown is the
 * temperature rise above the fixed (Dirichlet) or ambient (Robin) temperature. */
typedef enum {
    BKO_BC_DIRICHLET0 = 0, /* u = u0                                          */
    BKO_BC_ADIABATIC = 1,  /* zero normal flux                                */
    BKO_BC_ROBIN = 2       /* k du/dn + h (u - u_inf) = 0, h > 0              */
} bko_bc_kind;

typedef struct bko_operator *bko_op;

/* Preconditioner of the solves on an operator (bko_operator_set_precond).
 * The paper leaves it unstated; the default is none. */
typedef enum {
    BKO_PRECOND_NONE = 0,
    BKO_PRECOND_JACOBI = 1 /* diagonal (Jacobi) preconditioning, see below */
} bko_precond;

typedef struct {
    int iters;          /* inner block iterations, summed over refinements   */
    int refinements;    /* outer FP64 true-residual corrections (>= 1)        */
    int deflated;       /* search directions dropped as linearly dependent   */
    int status;         /* bko_status of the solve                           */
    double max_rel_res; /* max_j ||b_j - A x_j||_2 / ||b_j||_2, FP64, at exit */
    int x0_rejected;    /* initial-guess columns that fell back to zero       */
} bko_solve_info;

/* ------------------------------------------------------------------ build */

/* Library version string, e.g. "blockoa 0.1 gfx950". Static storage. */
const char *bko_version(void);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *bko_last_error(void);

/* ------------------------------------------------------- heat operator (A) */

/*
 * Bytes the caller must provide as coefficient storage for an nx x ny x nz
 * grid (Sec. II-B: the discretised operator A of Eq. (2)).  Storage holds
 * the diagonal and the three forward-face couplings per cell in FP64 and an
 * FP32 copy, the same four arrays of the diagonally scaled operator S A S
 * (S = diag(A)^(-1/2), for Jacobi preconditioning) in FP64 and FP32, and S
 * in FP64: 104 bytes per cell, each array 256-byte aligned.
 */
bko_status bko_operator_bytes(int nx, int ny, int nz, size_t *bytes);

/*
 * Discretise -div(k grad u) = q (Sec. II-A, Eq. (1), read in divergence form
 * so that A is symmetric positive definite) by cell-centred finite volumes
 * on an nx x ny x nz grid over lx x ly x lz (metres or any consistent unit):
 *   interior face a|b along spacing d :  w = 2 k_a k_b / ((k_a + k_b) d^2)
 *   Dirichlet-0 boundary face          :  w = 2 k_a / d^2
 *   adiabatic boundary face            :  w = 0
 *   Robin(h) boundary face             :  w = 1 / (d (d / (2 k_a) + 1 / h))
 *   (A x)_a = sum_b w_ab (x_a - x_b) + sum_boundary w x_a.
 * With nz == 1 and both z faces adiabatic the operator is the 5-point one.
 *
 *   k_cell_dev  device, N = nx*ny*nz doubles, conductivity per cell (> 0).
 *   bc          host, 6 face kinds ordered -x, +x, -y, +y, -z, +z.
 *   h           host, 6 film coefficients (read for BKO_BC_ROBIN faces, > 0).
 *   coeff_dev   device buffer of at least bko_operator_bytes() bytes,
 *               256-byte aligned; owned by the caller and must outlive *out.
 *   out         receives a handle (host metadata + coeff_dev).
 * Errors: BKO_EINVAL for bad sizes / kinds / h <= 0 on a Robin face / every
 * face adiabatic (A singular); BKO_ENOTSPD if any k is <= 0 or not finite
 * (checked on the device; the stream is synchronised).
 */
bko_status bko_assemble_heat_operator(int nx, int ny, int nz, double lx, double ly, double lz,
                                      const double *k_cell_dev, const int bc[6], const double h[6],
                                      void *coeff_dev, size_t coeff_bytes, void *stream,
                                      bko_op *out);

/* Grid of an operator: writes nx, ny, nz (any pointer may be NULL). */
bko_status bko_operator_dims(bko_op A, int *nx, int *ny, int *nz);

/*
 * Preconditioner of every later solve on A (bko_block_krylov_solve, batch
 * solves of chips on A, bko_cg_solve).  The paper does not state one
 * (Sec. V names PETSc without its options); BKO_PRECOND_NONE is the default.
 * BKO_PRECOND_JACOBI:
 *   block solve: the block iteration runs on the symmetrically scaled system
 *     (S A S) Y = S R, D = S Y, with S = diag(A)^(-1/2) (Jacobi applied on
 *     both sides, so the iterated operator stays symmetric positive
 *     definite); the FP64 correction loop still forms R = B - A X with the
 *     unscaled A and stops on the unscaled relative residual, so the
 *     solution meets the same tolerance as without preconditioning.
 *   per-sample CG: preconditioned CG with M = diag(A) (z = M^-1 r,
 *     rho = r'z), stopping on the unpreconditioned ||r|| <= tol ||b||.
 * Errors: BKO_EINVAL for a NULL handle or an unknown kind.
 */
bko_status bko_operator_set_precond(bko_op A, int kind);
bko_status bko_operator_get_precond(bko_op A, int *kind);

/*
 * Nonhomogeneous boundary data (Sec. II-A: Dirichlet u = u0, Robin ambient
 * u_inf, Mixed) by lifting: with face temperatures u_face[f] (the Dirichlet
 * value of a Dirichlet face, the ambient of a Robin face; ignored for
 * adiabatic faces) the temperature x solves A x = q + g, where A is the
 * operator assembled above and g_a = sum over the boundary faces of cell a
 * of w_face u_face (the same face weights as A).  Writes g (n FP64, device).
 * k_cell_dev: the conductivity the operator was assembled from.  Faces in
 * the order -x, +x, -y, +y, -z, +z.  Asynchronous.
 * Basis solutions of A X = Q + g 1^T combined with weights that sum to one
 * (bko_normalize_weights) keep the boundary data exactly; the power of a
 * field t is then A t - g (bko_add_column with alpha = -1).
 */
bko_status bko_boundary_source(bko_op A, const double *k_cell_dev, const double u_face[6], double *g, void *stream);

/* F[:, j] += alpha g for j < m (F n x m, ldf >= n; g n; FP64 device).  Asynchronous. */
bko_status bko_add_column(int n, int m, double *F, int ldf, const double *g, double alpha, void *stream);

/* Free the handle (host memory only; the coefficient buffer stays the caller's). */
bko_status bko_destroy_operator(bko_op A);

/* ------------------------------------------------------ basis solutions (X) */

/*
 * Workspace bytes for bko_block_krylov_solve with s right-hand sides and the
 * given inner compute dtype (BKO_F64 or BKO_F32).
 */
bko_status bko_block_krylov_workspace_bytes(bko_op A, int s, bko_dtype compute, size_t *bytes);

/*
 * Solve A X = B for s right-hand sides sharing A with one block Krylov
 * (block conjugate gradient) iteration (Sec. III-A, Eq. (4)).
 *
 * The block iteration keeps an orthonormal residual basis and SPD-solved
 * step matrices (a retooled block CG), and drops linearly dependent search
 * directions instead of breaking down.  Around it runs an FP64 correction
 * loop: R = B - A X is formed in FP64, the block iteration solves A D = R,
 * X += D, until max_j ||r_j|| / ||b_j|| <= tol (the per-column relative
 * residual norm used by the paper's tables, Sec. V).
 *
 *   compute = BKO_F64 : block iteration entirely in FP64.
 *   compute = BKO_F32 : block vectors and stencil products in FP32; the s x s
 *                       Gram matrices, their factorisations and the true
 *                       residual stay FP64 (mixed precision with FP64
 *                       iterative refinement).
 *   B (n x s, ldb >= n) FP64 device, X (n x s, ldx >= n) FP64 device output.
 *   X0 (ldx0 >= n) optional FP64 initial guess (e.g. a learned start); NULL
 *   means X0 = 0.  X0 may alias X (ldx0 == ldx).  Each column x0 is used as
 *   alpha x0 with alpha = x0'b / x0'A x0, the multiple of x0 closest to the
 *   solution in the A-norm (never further from it than the zero start); a
 *   column with alpha <= 0 or not finite falls back to the zero start and is
 *   counted in info->x0_rejected.
 *   tol > 0, max_iter >= 1 caps the total inner iterations.
 *   work / work_bytes: caller workspace (bko_block_krylov_workspace_bytes),
 *   256-byte aligned, contents need not be initialised.
 *   info (host, may be NULL) receives iteration counts and the final FP64
 *   relative residual.
 * Returns BKO_OK on convergence, BKO_ENOCONV if max_iter was reached (X
 * holds the last iterate and info its residual), BKO_EBREAKDOWN if every
 * direction deflated above tol.  Synchronises the stream.
 */
bko_status bko_block_krylov_solve(bko_op A, int s, const double *B, int ldb, double *X, int ldx,
                                  const double *X0, int ldx0, bko_dtype compute, double tol,
                                  int max_iter, void *work, size_t work_bytes,
                                  bko_solve_info *info, void *stream);

/* ------------------------------------------------- batches of chips */

typedef struct bko_batch_plan *bko_batch;

/*
 * A batch of chips solved together: the chip index j of Eq. (4) (Sec. III-A)
 * runs over the batch, each chip with its own operator and grid, all with
 * the same s.  Every kernel of a block iteration covers all chips in one
 * launch (a workgroup table maps workgroups to chips), chips that have
 * converged drop out at the next launch, and the iteration chunks between
 * convergence checks are captured into HIP graphs and replayed when the
 * stream is not the null stream.
 *   ops   host array of nchips operator handles (they must outlive the plan).
 *   m     host array of nchips field counts M_c for bko_batch_run (0: no
 *         fields for that chip), or NULL for a plan that only solves.
 *   dt    host array of four dtypes: dt[0] the block iteration (BKO_F64, or
 *         BKO_F32 with FP64 Gram matrices, factorisations and refinement),
 *         dt[1] the combination's arithmetic (as bko_combine's compute),
 *         dt[2] the storage type of T, dt[3] that of F.  The operator action
 *         computes in FP64 when T and F are both FP64, else with FP32
 *         coefficients and accumulation.
 * The plan holds host metadata only.
 */
bko_status bko_batch_plan_create(int nchips, const bko_op *ops, int s, const int *m, const bko_dtype dt[4],
                                 bko_batch *out);
bko_status bko_batch_plan_destroy(bko_batch plan);

/* Workspace bytes of a batch solve or run (caller-owned, 256-byte aligned). */
bko_status bko_batch_workspace_bytes(bko_batch plan, size_t *bytes);

/*
 * Autotuner: times the row kernels for each candidate number of 256-row
 * tiles per workgroup (1, 2, 4, 8: each chip then runs ceil(tiles / t)
 * workgroups, and its Gram reductions sum as many partials), over the whole
 * batch and over its largest chip alone (the tail of a batch solve), and
 * keeps the fastest in the plan.  The workspace contents are overwritten.
 * tiles_per_wg (host, may be NULL) receives the choice.  bko_batch_solve
 * tunes on its first call if this was not called.  Synchronises the stream.
 */
bko_status bko_batch_tune(bko_batch plan, void *work, size_t work_bytes, int *tiles_per_wg, void *stream);

/*
 * Solve A_c X_c = B_c for every chip c of the plan (semantics of
 * bko_block_krylov_solve per chip).  B, X, X0 are host arrays of nchips
 * device pointers (n_c x s, column major, leading dimensions in ldb, ldx,
 * ldx0); X0 may be NULL, or hold NULL for a zero start of that chip.
 * infos (host, may be NULL) receives nchips records.  Returns BKO_OK when
 * every chip converged, else the first failing chip's status (each chip's
 * own status is in infos).  Synchronises the stream.
 */
bko_status bko_batch_solve(bko_batch plan, const double *const *B, const int *ldb, double *const *X,
                           const int *ldx, const double *const *X0, const int *ldx0, double tol,
                           int max_iter, void *work, size_t work_bytes, bko_solve_info *infos,
                           void *stream);

/*
 * The whole path for every chip of the plan (Sec. III): the basis solutions
 * A_c X_c = B_c (as bko_batch_solve, zero start), then T_c = X_c C_c
 * (Sec. III-B, Eq. (5)) for every chip in one grouped combination launch,
 * then F_c = A_c T_c of the T written (Sec. III-C, Eq. (6)) for every chip
 * in one grouped operator-action launch (chips whose rows are not a whole
 * number of 16-byte vectors, or whose views are not 16-byte aligned, get an
 * operator-action launch of their own).  Host arrays of nchips device
 * pointers: B, X (n_c x s FP64, ldb, ldx >= n_c), C (s x M_c FP64,
 * ldc >= s: column j holds field j's weights), T (n_c x M_c of dt[2],
 * ldt >= n_c), F (n_c x M_c of dt[3], ldf >= n_c, not overlapping T).  On
 * the plan's first run the grouped launches' knobs (the combination's fields
 * per workgroup, the operator action's tile height) are chosen by timing a
 * few candidates on these outputs, and cached for the device architecture
 * and batch shape.  The outputs are written even when a chip does not
 * converge (its X is the last iterate); the return value is the solve's.
 * infos as for bko_batch_solve.  Synchronises the stream.
 */
bko_status bko_batch_run(bko_batch plan, const double *const *B, const int *ldb, double *const *X, const int *ldx,
                         const double *const *C, const int *ldc, void *const *T, const int *ldt, void *const *F,
                         const int *ldf, double tol, int max_iter, void *work, size_t work_bytes,
                         bko_solve_info *infos, void *stream);

/* The output knobs bko_batch_run chose (host; -1 before the first run): the
 * cap on the operator action's tile height (0: the kernel's full height)
 * and the combination's fields per workgroup (0: the launcher's rule). */
bko_status bko_batch_output_tuning(bko_batch plan, int *tile_rows_cap, int64_t *fields_per_wg);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * block solve as bko_block_krylov_solve, same arguments and results, with
 * the workspace taken from scratch memory the library holds itself
 * (BKO_NOALLOC_SCRATCH_BYTES per device, held until the process ends).
 * Calls no hipMalloc or hipFree.  A solve whose workspace
 * (bko_block_krylov_workspace_bytes) exceeds the scratch returns BKO_EINVAL
 * and launches nothing.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one GPU (other threads, other streams) race and must
 * be serialised by the caller.  The scratch keeps the last call's contents;
 * the solve initialises everything it reads.  Synchronises the stream.
 */
#define BKO_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
bko_status bko_block_krylov_solve_noalloc(bko_op A, int s, const double *B, int ldb, double *X, int ldx,
                                          const double *X0, int ldx0, bko_dtype compute, double tol, int max_iter,
                                          bko_solve_info *info, void *stream);

/* ------------------------------------------- per-sample CG (the baseline) */

/* Workspace bytes for bko_cg_solve with m right-hand sides. */
bko_status bko_cg_workspace_bytes(bko_op A, int m, size_t *bytes);

/*
 * The direct method the paper compares against (Sec. III, the per-sample
 * baseline of Table 1): an independent conjugate gradient solve of
 * A x_j = b_j for each of m columns, without sharing a Krylov space.  Columns
 * are batched so one stencil launch serves them all, but every column has
 * its own step lengths and stops on its own recurrence residual
 * ||r_j|| <= tol ||b_j|| (x_0 = 0, FP64, no preconditioner).
 *   B (n x m, ldb >= n) and X (n x m, ldx >= n) FP64 device.
 *   iters (host, may be NULL) receives m per-column iteration counts.
 *   info (host, may be NULL): iters = the largest column count, max_rel_res
 *   the largest FP64 true relative residual at exit.
 * Returns BKO_ENOCONV if a column is still running after max_iter
 * iterations.  Synchronises the stream.
 */
bko_status bko_cg_solve(bko_op A, int m, const double *B, int ldb, double *X, int ldx, double tol,
                        int max_iter, void *work, size_t work_bytes, int *iters, bko_solve_info *info,
                        void *stream);

/* ------------------------------------------------- combination (T = X C) */

/*
 * T = X C: M temperature fields as combinations of s basis solutions
 * (Sec. III-B, Eq. (5), with raw weights; normalising the weights is the
 * caller's choice of C).  X is n x s (ldx >= n), C is s x m (ldc >= s),
 * T is n x m (ldt >= n).  Inputs of any dtype are converted in-register to
 * the compute dtype: BKO_F64 (FP64 matrix cores), BKO_F32 (FP32 matrix
 * cores, FP32 accumulate) or BKO_BF16 (inputs rounded to BF16, FP32
 * accumulate).  T is written in t_t.  Asynchronous.
 */
bko_status bko_combine(int n, int s, int m, const void *X, int ldx, bko_dtype x_t,
                       const void *C, int ldc, bko_dtype c_t, void *T, int ldt, bko_dtype t_t,
                       bko_dtype compute, void *stream);

/*
 * Noise of Eq. (5) (Sec. III-B; the paper's default draws it uniformly from
 * (-0.01, 0.01) at each grid point, Sec. V-B): a counter-based generator,
 * Philox4x32-10 (Salmon et al., SC 2011), keyed by seed and counting
 * (cell, global field index), so the value at (field f, cell a) does not
 * depend on how the fields are split over calls.  With 52 bits u of the
 * first two output words: uniform = amplitude ((2u + 1) 2^-52 - 1) on
 * (-amplitude, amplitude); Gaussian = amplitude sqrt(-2 ln x1) cos(2 pi x2)
 * (Box-Muller, x = (u + 1/2) 2^-52 from words 0-1 and 2-3).  The noise is
 * added to every cell: the boundary models live in A, so the fields keep
 * their boundary conditions.
 */
typedef enum { BKO_NOISE_NONE = 0, BKO_NOISE_UNIFORM = 1, BKO_NOISE_GAUSSIAN = 2 } bko_noise_kind;
typedef struct {
    int kind;              /* bko_noise_kind                                   */
    double amplitude;      /* half-width (uniform) or standard deviation        */
    unsigned long long seed;         /* generator key                          */
    unsigned long long field_offset; /* global index of the call's field 0     */
} bko_noise;

/*
 * T = X C + E (FP64): the combination of Eq. (5) with its noise term.  X
 * n x s (ldx >= n), C s x m (ldc >= s), T n x m (ldt >= n); noise may be
 * NULL (no noise).  The operator action of these fields is then
 * bko_apply_operator on T (F = A T covers A E).  Asynchronous.
 */
bko_status bko_combine_noisy(int n, int s, int m, const double *X, int ldx, const double *C, int ldc, double *T,
                             int ldt, const bko_noise *noise, void *stream);

/* E (n x m, lde >= n, FP64 device) = the noise alone, as added by
 * bko_combine_noisy.  Asynchronous. */
bko_status bko_noise_fill(int n, int m, double *E, int lde, const bko_noise *noise, void *stream);

/*
 * The normalised weights of Eq. (5), alpha_i = mu_i / sum_j mu_j, in place
 * on C (s x m, ldc >= s, FP64 device; column j holds field j's mu), the sum
 * taken in index order.  The sum of s standard normals can be close to
 * zero: a field with |sum| < min_abs_sum keeps its mu and gets flags[j] = 1
 * (flags: m ints, device, written for every field; the caller draws new mu
 * for the flagged fields and calls again).  Asynchronous.
 */
bko_status bko_normalize_weights(int s, int m, double *C, int ldc, double min_abs_sum, int *flags, void *stream);

/* Workspace bytes of bko_combine_apply (an n x s FP64 block). */
bko_status bko_combine_apply_workspace_bytes(bko_op A, int s, size_t *bytes);

/*
 * The temperature fields and their operator action in one pass over the
 * fields, FP64: T = X C (Sec. III-B, Eq. (5)) and F = A T (Sec. III-C,
 * Eq. (6)) computed as F = (A X) C, which equals A (X C) exactly in exact
 * arithmetic and to rounding in FP64 (every pair then satisfies
 * ||A t - f|| <= a few ulp of |A||X||C|).  The s columns of A X are formed
 * first (one stencil product over s columns, in the workspace), then one
 * kernel writes both outputs, so T is never read back.  X n x s (ldx >= n),
 * C s x m (ldc >= s), T and F n x m (ldt, ldf >= n), all FP64 device; T, F
 * must not overlap X or each other.  work: caller workspace of
 * bko_combine_apply_workspace_bytes, 256-byte aligned.  Asynchronous.
 */
bko_status bko_combine_apply(bko_op A, int s, int m, const double *X, int ldx, const double *C, int ldc, double *T,
                             int ldt, double *F, int ldf, void *work, size_t work_bytes, void *stream);

/* ----------------------------------------------- operator action (F = A T) */

/*
 * F = A T for m fields (Sec. III-C, Eq. (6)): one matrix-free stencil
 * product per field, no solve.  T is n x m (ldt >= n) in t_t, F is n x m
 * (ldf >= n) in f_t.  compute = BKO_F64 uses the FP64 coefficients and
 * FP64 accumulation; BKO_F32 (or BKO_BF16) uses the FP32 coefficients and
 * FP32 accumulation.  T and F must not overlap.  Asynchronous.
 */
bko_status bko_apply_operator(bko_op A, int m, const void *T, int ldt, bko_dtype t_t, void *F,
                              int ldf, bko_dtype f_t, bko_dtype compute, void *stream);

/*
 * dst = src, `bytes` bytes of device memory, one 16-byte vector load and
 * store per thread (the library's reference for achievable HBM bandwidth:
 * every HBM-bound kernel of the path reads and writes whole fields with
 * 16-byte vector accesses).
 * Both pointers 16-byte aligned, bytes a multiple of 16, no overlap;
 * otherwise BKO_EINVAL.  Asynchronous.
 */
bko_status bko_copy(void *dst, const void *src, size_t bytes, void *stream);

/*
 * Which operator-action kernel bko_apply_operator would run for these
 * arguments, compute included (pointers are compared for alignment only,
 * never read):
 * *tile_rows = the rows per tile of the z-marching LDS-tiled kernel
 * (full-width row tiles with a one-row halo, 16-byte vector access), or 0
 * when the per-cell kernel takes the call (rows that are not a whole number
 * of 16-byte vectors, views not 16-byte aligned, or tiles too short to pay
 * for their halo).  Host only, no launch.
 */
bko_status bko_apply_operator_tiling(bko_op A, int m, const void *T, int ldt, bko_dtype t_t, const void *F, int ldf,
                                     bko_dtype f_t, bko_dtype compute, int *tile_rows);

/*
 * Fused residual form used by the correction loop: R = B - A X in FP64
 * (B, X, R n x m, FP64).  R may alias B.  Asynchronous.
 */
bko_status bko_residual(bko_op A, int m, const double *B, int ldb, const double *X, int ldx,
                        double *R, int ldr, void *stream);

/* ------------------------------------------------ learned initial guess */

/*
 * A 4-level convolutional encoder-decoder that predicts the basis solutions
 * of a chip from its power maps, conductivity and film coefficient; its
 * output is the X0 argument of the block solve (Sec. III-A starts the block
 * iteration from any initial block; zero start is the fallback).  Not part
 * of the paper.  Tensors are FP32, layout (N, C, H, W), device memory.
 *
 * Layers (3 x 3 "same" convolutions, bias, ReLU, except the last):
 *   0,1 Cin->w1->w1 at H | 2,3 pool: w1->w2->w2 at H/2 | 4,5 pool: w2->w3->w3
 *   at H/4 | 6,7 pool: w3->w4->w4 at H/8 | 8,9 [up(7), out 5]: w4+w3->w3->w3
 *   | 10,11 [up(9), out 3]: w3+w2->w2->w2 | 12,13 [up(11), out 1]:
 *   w2+w1->w1->w1 | 14 1 x 1 w1->Cout, no ReLU;
 * w1 = base, w2 = 2 base, w3 = w4 = 4 base; pool = 2 x 2 average, up =
 * nearest 2x, [a, b] = channel concatenation.  Flat parameters: per layer in
 * this order, filter (Cout, Cin, K, K) row-major then bias (Cout).
 *
 * State buffer (caller-owned, 256-byte aligned, bko_unet_sizes bytes):
 * FP32 parameters [nparams], FP32 gradients [nparams], Adam first and
 * second moments [nparams each], then the BF16 copy of the parameters that
 * every convolution reads (FP32 accumulation).  The workspace holds the
 * activations of up to max_batch samples.
 */
typedef struct bko_unet *bko_net;

bko_status bko_unet_create(int cin, int cout, int base, int height, int width, int max_batch, bko_net *out);
bko_status bko_unet_destroy(bko_net net);
bko_status bko_unet_sizes(bko_net net, int64_t *nparams, size_t *state_bytes, size_t *work_bytes);

/* Load FP32 parameters (device, nparams), clear the Adam state and step count. */
bko_status bko_unet_set_params(bko_net net, void *state, const float *params, void *stream);

/* y (n, Cout, H, W) = network(x (n, Cin, H, W)), 1 <= n <= max_batch. Asynchronous. */
bko_status bko_unet_forward(bko_net net, void *state, void *work, const float *x, int n, float *y, void *stream);

/*
 * The same network for inference with every convolution on the BF16 matrix
 * cores: each convolution's input is rounded to BF16 (nearest even) before
 * the products (the parameters are the BF16 copy, as in bko_unet_forward),
 * FP32 accumulation, bias and ReLU.  One BF16 rounding per layer (relative
 * 2^-9 each) makes it differ from bko_unet_forward by about 1e-2 of ||y||
 * over the fifteen layers; used for the learned start's initial guess, which
 * the block solve then refines.  Same arguments and errors as
 * bko_unet_forward.  Asynchronous.
 */
bko_status bko_unet_infer(bko_net net, void *state, void *work, const float *x, int n, float *y, void *stream);

/*
 * Forward pass, loss = mean over all n Cout H W outputs of (y - target)^2,
 * and its gradient with respect to every parameter into the state's gradient
 * block.  loss (host, may be NULL) receives the loss and then the call
 * synchronises the stream; with NULL it is asynchronous.
 */
bko_status bko_unet_gradient(bko_net net, void *state, void *work, const float *x, const float *target, int n,
                             float *loss, void *stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on the state's
 * gradients; refreshes the BF16 copy.  Asynchronous. */
bko_status bko_unet_adam_step(bko_net net, void *state, float lr, void *stream);

/*
 * Building blocks, exposed for tests: one convolution (mode 0 reads A (N,
 * Ca, H, W); mode 1 the 2 x 2 average of A (N, Ca, 2H, 2W); mode 2 the
 * concatenation of A (N, Ca, H/2, W/2) upsampled and B (N, Cb, H, W)), with
 * BF16 filters wgt (Co, Ca + Cb, K, K), or with transposed != 0 the flipped,
 * transposed filters of a layer (Ca + Cb, Co, K, K) (the input gradient);
 * bias may be NULL.  And the filter / bias gradient of such a convolution
 * for output gradient g (N, Co, H, W) into gw (Co, Ca + Cb, K, K) and gb
 * (Co), with a work buffer of bko_nn_wgrad_work_floats floats.
 */
bko_status bko_nn_conv2d(const float *A, int Ca, const float *B, int Cb, int mode, int N, int H, int W, int Co, int K,
                         const uint16_t *wgt, int transposed, const float *bias, float *out, int relu, void *stream);
size_t bko_nn_wgrad_work_floats(int N, int H, int W, int Ci, int Co, int K);
bko_status bko_nn_conv2d_wgrad(const float *A, int Ca, const float *B, int Cb, int mode, const float *g, int N, int H,
                               int W, int Co, int K, float *work, float *gw, float *gb, void *stream);

/*
 * Network input of m fields of one chip: channels [0, nz) = F[:, j] /
 * scale[j] as nz planes of ny x nx (the field layout itself), [nz, 2 nz) =
 * (log k - kmu) / ksig per layer, 2 nz = hval everywhere; scale[j] =
 * ||F[:, j]||_2 / sqrt(n), the RMS value (FP64; 0 gives zero planes).  x is
 * (m, 2 nz + 1, ny, nx).
 */
bko_status bko_lstart_pack(int nx, int ny, int nz, const double *F, int ldf, int m, const double *k_cell, float kmu,
                           float ksig, float hval, double *scale, float *x, void *stream);
/*
 * sweeps damped Jacobi sweeps X <- X + omega (B - A X) / diag(A) (FP64, m
 * columns, 0 < omega < 2): damps the high-frequency error of an initial
 * guess (a learned X0 is accurate in its smooth part, and the block solve
 * converges on the rest).  work: n x m FP64 scratch (ldw >= n).  Asynchronous.
 */
bko_status bko_jacobi_smooth(bko_op A, int m, const double *B, int ldb, double *X, int ldx, double *work, int ldw,
                             int sweeps, double omega, void *stream);

/* Training target t (m, n) = T[:, j] / (scale[j] gain). */
bko_status bko_lstart_pack_target(int n, const double *T, int ldt, int m, const double *scale, double gain, float *t,
                                  void *stream);
/* X0[:, j] = y (m, n)[j] * scale[j] * gain (FP64 initial guess). */
bko_status bko_lstart_unpack(int n, const float *y, int m, const double *scale, double gain, double *X0, int ldx,
                             void *stream);

/* ---------------------------------------------------- kernel timing hooks */

/*
 * Optional per-kernel timing: `mask` selects kernel families (bit f = family
 * f, 0 = off).  For a selected family the library takes a HIP event pair per
 * launch on the launch stream and accumulates the elapsed time when queried
 * (which synchronises): the block-solve kernels take the pair inside their
 * own dispatch (kernel begin and end, what a kernel trace records); the
 * operator action, combine and per-sample CG stencil bracket their launch
 * with stream markers.  bko_timing_set_stride(k) times one launch in every
 * k of each family (k >= 1, default 1; resets the per-family counters), so
 * that the events' own cost stays small in a timed loop; bko_timing_query
 * then counts the timed launches only.
 * Families: 0 = operator action, 1 = combine, 2 = Gram partials, 3 = block
 * update W, 4 = Gram reduction (+ s x s factorisation for s > 32), 5 =
 * block-solve stencil product, 6 = FP64 residual, 7 = block update D, Q, P.
 * Timed launches are not captured into graphs.  Used to report per-kernel
 * bandwidth.
 */
bko_status bko_timing_enable(int mask);
bko_status bko_timing_set_stride(int every);
bko_status bko_timing_query(int family, int *launches, double *total_ms);
bko_status bko_timing_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* BLOCKOA_H */
