/*
 * CPU oracle for the block Krylov + operator action data path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct FP64
 * reference.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * What it computes (the plain definitions the method reaches):
 *   - the discretised steady heat operator A as an assembled CSR matrix
 *     (paper Sec. II-A, Eq. (1) with its Dirichlet / Robin boundary models,
 *     read in divergence form so that A is symmetric positive definite, as the
 *     paper's "sparse symmetric matrices" of Sec. V-A require);
 *   - X = A^{-1} B by unpreconditioned conjugate gradients, one right-hand side
 *     at a time, from x0 = 0 (the paper's direct solution method, Sec. II-D,
 *     and its CG baseline, Sec. V-A);
 *   - the same with diagonal (Jacobi) preconditioning, M = diag(A), stopping
 *     on the unpreconditioned residual (the paper leaves the preconditioner
 *     unstated; this defines the optional Jacobi mode of the baseline);
 *   - T = X C by plain loops (Sec. III-B, Eq. (5) with raw weights);
 *   - F = A T by CSR matrix-vector products (Sec. III-C, Eq. (6)).
 *
 * Discretisation (cell-centred finite volumes on an nx x ny x nz grid over
 * lx x ly x lz, cell index n = i + nx*(j + ny*l)):
 *   interior face between cells a, b along an axis of spacing d:
 *       w = 2 k_a k_b / ((k_a + k_b) d^2)          (series conduction)
 *   boundary face of cell a:
 *       Dirichlet-0 : w = 2 k_a / d^2              (half-cell conduction)
 *       adiabatic   : w = 0
 *       Robin(h)    : w = 1 / (d (d / (2 k_a) + 1 / h))
 *   (A x)_a = sum_b w_ab (x_a - x_b) + sum_faces w_face x_a.
 * Unknowns are the temperature rise above the boundary / ambient temperature.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_DIRICHLET0 = 0, ORC_ADIABATIC = 1, ORC_ROBIN = 2 };

static double face_boundary(int kind, double ka, double d, double h)
{
    if (kind == ORC_DIRICHLET0) return 2.0 * ka / (d * d);
    if (kind == ORC_ROBIN) return 1.0 / (d * (d / (2.0 * ka) + 1.0 / h));
    return 0.0;
}

static double face_interior(double ka, double kb, double d)
{
    return 2.0 * ka * kb / ((ka + kb) * d * d);
}

/* Upper bound on the number of stored entries: 7 per row. */
int64_t orc_nnz_bound(int nx, int ny, int nz)
{
    return 7 * (int64_t)nx * ny * nz;
}

/*
 * Assemble A in CSR form.  Columns within a row are stored in ascending order
 * (neighbours below and the diagonal in index order).  Returns the number of
 * stored entries, or -1 on bad input.
 */
int64_t orc_assemble_csr(int nx, int ny, int nz, double lx, double ly, double lz,
                         const double *k, const int *bc, const double *h,
                         int64_t *rowptr, int32_t *col, double *val)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const double d[3] = {lx / nx, ly / ny, lz / nz};
    const int n3[3] = {nx, ny, nz};
    const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
    const int64_t N = (int64_t)nx * ny * nz;
    int64_t pos = 0;
    for (int64_t a = 0; a < N; ++a) {
        int idx[3];
        idx[0] = (int)(a % nx);
        idx[1] = (int)((a / nx) % ny);
        idx[2] = (int)(a / ((int64_t)nx * ny));
        rowptr[a] = pos;
        double diag = 0.0;
        /* neighbour entries, gathered then emitted in ascending column order */
        int64_t nbr_col[6];
        double nbr_w[6];
        int nn = 0;
        for (int ax = 0; ax < 3; ++ax) {
            /* minus side */
            if (idx[ax] > 0) {
                int64_t b = a - stride[ax];
                double w = face_interior(k[a], k[b], d[ax]);
                nbr_col[nn] = b; nbr_w[nn] = w; ++nn;
                diag += w;
            } else {
                diag += face_boundary(bc[2 * ax], k[a], d[ax], h[2 * ax]);
            }
            /* plus side */
            if (idx[ax] < n3[ax] - 1) {
                int64_t b = a + stride[ax];
                double w = face_interior(k[a], k[b], d[ax]);
                nbr_col[nn] = b; nbr_w[nn] = w; ++nn;
                diag += w;
            } else {
                diag += face_boundary(bc[2 * ax + 1], k[a], d[ax], h[2 * ax + 1]);
            }
        }
        /* insertion sort of the (at most six) neighbours, then place the diagonal */
        for (int i = 1; i < nn; ++i) {
            int64_t c = nbr_col[i]; double w = nbr_w[i]; int j = i - 1;
            while (j >= 0 && nbr_col[j] > c) { nbr_col[j + 1] = nbr_col[j]; nbr_w[j + 1] = nbr_w[j]; --j; }
            nbr_col[j + 1] = c; nbr_w[j + 1] = w;
        }
        int placed = 0;
        for (int i = 0; i < nn; ++i) {
            if (!placed && nbr_col[i] > a) { col[pos] = (int32_t)a; val[pos] = diag; ++pos; placed = 1; }
            col[pos] = (int32_t)nbr_col[i]; val[pos] = -nbr_w[i]; ++pos;
        }
        if (!placed) { col[pos] = (int32_t)a; val[pos] = diag; ++pos; }
    }
    rowptr[N] = pos;
    return pos;
}

/* y = A x */
void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y)
{
    for (int64_t r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) acc += val[p] * x[col[p]];
        y[r] = acc;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

/*
 * Conjugate gradients for one right-hand side from x = 0, stopping when the
 * recurrence residual satisfies ||r|| <= tol ||b|| or after maxit iterations.
 * On return relres holds the TRUE relative residual ||b - A x|| / ||b||.
 * Returns the number of iterations taken.  scratch must hold 3n doubles.
 */
int orc_cg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
           const double *b, double *x, double tol, int maxit, double *relres, double *scratch)
{
    double *r = scratch, *p = scratch + n, *q = scratch + 2 * n;
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    const double bnorm = sqrt(dot(n, b, b));
    int it = 0;
    if (bnorm == 0.0) { *relres = 0.0; return 0; }
    double rr = dot(n, r, r);
    while (it < maxit && sqrt(rr) > tol * bnorm) {
        orc_spmv(n, rowptr, col, val, p, q);
        const double alpha = rr / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        const double rr_new = dot(n, r, r);
        const double beta = rr_new / rr;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        ++it;
    }
    orc_spmv(n, rowptr, col, val, x, q);
    double res = 0.0;
    for (int64_t i = 0; i < n; ++i) { const double e = b[i] - q[i]; res += e * e; }
    *relres = sqrt(res) / bnorm;
    return it;
}

/*
 * Independent CG solves for s right-hand sides (columns of B, leading
 * dimension ldb), one column per thread.  nthreads <= 0 means the OpenMP
 * default.
 */
void orc_cg_many(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                 int s, const double *B, int64_t ldb, double *X, int64_t ldx,
                 double tol, int maxit, int *iters, double *relres, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *scratch = (double *)malloc(sizeof(double) * 3 * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int j = 0; j < s; ++j)
            iters[j] = orc_cg(n, rowptr, col, val, B + j * ldb, X + j * ldx, tol, maxit,
                              &relres[j], scratch);
        free(scratch);
    }
    (void)nthreads;
}

/*
 * Preconditioned CG with M^{-1} = diag(minv) for one right-hand side from
 * x = 0: z = M^{-1} r, rho = r.z, alpha = rho / p.Ap, x += alpha p,
 * r -= alpha Ap, p = z' + (rho' / rho) p; stops when the unpreconditioned
 * recurrence residual satisfies ||r|| <= tol ||b|| or after maxit
 * iterations.  relres and the return value as for orc_cg.  scratch must
 * hold 4n doubles.
 */
int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, const double *minv,
            const double *b, double *x, double tol, int maxit, double *relres, double *scratch)
{
    double *r = scratch, *p = scratch + n, *q = scratch + 2 * n, *z = scratch + 3 * n;
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; z[i] = minv[i] * r[i]; p[i] = z[i]; }
    const double bnorm = sqrt(dot(n, b, b));
    int it = 0;
    if (bnorm == 0.0) { *relres = 0.0; return 0; }
    double rho = dot(n, r, z);
    while (it < maxit && sqrt(dot(n, r, r)) > tol * bnorm) {
        orc_spmv(n, rowptr, col, val, p, q);
        const double alpha = rho / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; z[i] = minv[i] * r[i]; }
        const double rho_new = dot(n, r, z);
        const double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
        ++it;
    }
    orc_spmv(n, rowptr, col, val, x, q);
    double res = 0.0;
    for (int64_t i = 0; i < n; ++i) { const double e = b[i] - q[i]; res += e * e; }
    *relres = sqrt(res) / bnorm;
    return it;
}

/* Jacobi-preconditioned CG (M = diag(A)) per column, one column per thread. */
void orc_pcg_many(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  int s, const double *B, int64_t ldb, double *X, int64_t ldx,
                  double tol, int maxit, int *iters, double *relres, int nthreads)
{
    double *minv = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        double d = 0.0;
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p)
            if (col[p] == r) d += val[p];
        minv[r] = 1.0 / d;
    }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *scratch = (double *)malloc(sizeof(double) * 4 * (size_t)n);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int j = 0; j < s; ++j)
            iters[j] = orc_pcg(n, rowptr, col, val, minv, B + j * ldb, X + j * ldx, tol, maxit,
                               &relres[j], scratch);
        free(scratch);
    }
    free(minv);
    (void)nthreads;
}

/* T = X C (n x s times s x m, all column-major) by plain loops. */
void orc_gemm(int64_t n, int s, int64_t m, const double *X, int64_t ldx,
              const double *C, int64_t ldc, double *T, int64_t ldt, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
    for (int64_t f = 0; f < m; ++f) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int kk = 0; kk < s; ++kk) acc += X[i + kk * ldx] * C[kk + f * ldc];
            T[i + f * ldt] = acc;
        }
    }
    (void)nthreads;
}

/* F = A T, one CSR product per column. */
void orc_apply_many(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                    int64_t m, const double *T, int64_t ldt, double *F, int64_t ldf, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
    for (int64_t f = 0; f < m; ++f) orc_spmv(n, rowptr, col, val, T + f * ldt, F + f * ldf);
    (void)nthreads;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
