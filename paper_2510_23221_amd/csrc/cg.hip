// Per-sample conjugate gradient: the direct data-generation method the paper
// compares against (Sec. III, the baseline of Table 1), one independent
// Hestenes-Stiefel CG per right-hand side, batched as columns so that the
// stencil product of every active column shares one launch.  Each column has
// its own step lengths and stops on its own recurrence residual:
//     x_0 = 0, r_0 = p_0 = b
//     alpha = (r^T r) / (p^T A p) ; x += alpha p ; r -= alpha A p
//     beta  = (r'^T r') / (r^T r) ; p  = r' + beta p
// until ||r|| <= tol ||b||.  FP64 throughout.  With the operator's Jacobi
// preconditioner (M = diag(A)) it is preconditioned CG: z = M^-1 r,
// rho = r^T z, beta = rho' / rho, p = z' + beta p, with the same stop test
// on the unpreconditioned residual.
//
// Kernels per iteration (one stream, no host round trip): stencil A p; column
// dot partials p^T A p; per-column alpha; x, r update with r^T r partials;
// per-column beta and the stop test; p update.  Columns that have stopped are
// skipped by the vector kernels (their stencil product is still formed, since
// the stencil launch covers the whole block).
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

constexpr int kCgThreads = 256;
constexpr int kRowsPerChunk = 4096;

enum CgCtrl { kRemaining = 0 };

struct CgWork {
    int64_t ldw;
    double *R, *P, *AP;
    double *part;     // [chunks][m] column partial sums
    double *part2;    // [chunks][m] partial sums of r^T M^-1 r (preconditioned)
    double *rho, *alpha, *beta, *th2;
    int *done, *iters, *ctrl;
    int chunks;
    size_t bytes;
};

inline CgWork carve_cg(void *base, int64_t n, int m)
{
    CgWork w{};
    w.ldw = static_cast<int64_t>(align_up(static_cast<size_t>(n), 256));
    w.chunks = static_cast<int>((n + kRowsPerChunk - 1) / kRowsPerChunk);
    char *p = static_cast<char *>(base);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *q = p + o;
        o = align_up(o + bytes, 256);
        return q;
    };
    const size_t blk = sizeof(double) * static_cast<size_t>(w.ldw) * m;
    w.R = reinterpret_cast<double *>(take(blk));
    w.P = reinterpret_cast<double *>(take(blk));
    w.AP = reinterpret_cast<double *>(take(blk));
    w.part = reinterpret_cast<double *>(take(sizeof(double) * static_cast<size_t>(w.chunks) * m));
    w.part2 = reinterpret_cast<double *>(take(sizeof(double) * static_cast<size_t>(w.chunks) * m));
    w.rho = reinterpret_cast<double *>(take(sizeof(double) * m));
    w.alpha = reinterpret_cast<double *>(take(sizeof(double) * m));
    w.beta = reinterpret_cast<double *>(take(sizeof(double) * m));
    w.th2 = reinterpret_cast<double *>(take(sizeof(double) * m));
    w.done = reinterpret_cast<int *>(take(sizeof(int) * m));
    w.iters = reinterpret_cast<int *>(take(sizeof(int) * m));
    w.ctrl = reinterpret_cast<int *>(take(sizeof(int) * 64));
    w.bytes = o;
    return w;
}

__device__ inline double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kCgThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    return sh[0];
}

// part[c * m + j] = sum over rows of chunk c of a_j * b_j, times scale^2
// per row when scale is given (grid: chunks x m)
__global__ __launch_bounds__(kCgThreads) void coldot_kernel(const double *__restrict__ a, int64_t lda,
                                                            const double *__restrict__ b, int64_t ldb, int64_t n,
                                                            int m, double *__restrict__ part,
                                                            const int *__restrict__ done,
                                                            const double *__restrict__ scale = nullptr)
{
    __shared__ double sh[kCgThreads];
    const int j = blockIdx.y;
    if (done && done[j]) return;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRowsPerChunk;
    const int64_t r1 = min(n, r0 + kRowsPerChunk);
    const double *aj = a + j * lda, *bj = b + j * ldb;
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kCgThreads) {
        const double w = scale ? scale[r] * scale[r] : 1.0;
        acc = fma(aj[r] * w, bj[r], acc);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[static_cast<int64_t>(blockIdx.x) * m + j] = t;
}

// Sum of the chunk partials of column j in chunk order.
__device__ inline double sum_parts(const double *part, int chunks, int m, int j)
{
    double t = 0.0;
    for (int c = 0; c < chunks; ++c) t += part[static_cast<int64_t>(c) * m + j];
    return t;
}

// alpha_j = rho_j / (p_j^T A p_j) for active columns
__global__ void cg_alpha_kernel(const double *__restrict__ part, int chunks, int m, const double *__restrict__ rho,
                                double *__restrict__ alpha, const int *__restrict__ done)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || done[j]) return;
    const double pap = sum_parts(part, chunks, m, j);
    alpha[j] = pap > 0.0 ? rho[j] / pap : 0.0;
}

// x += alpha p ; r -= alpha A p ; part = chunk sums of r^T r and, with a
// preconditioner (scale^2 = M^-1), part2 = chunk sums of r^T M^-1 r
// (grid: chunks x m)
__global__ __launch_bounds__(kCgThreads) void cg_update_kernel(double *__restrict__ X, int64_t ldx,
                                                               double *__restrict__ R, const double *__restrict__ P,
                                                               const double *__restrict__ AP, int64_t ldw, int64_t n,
                                                               int m, const double *__restrict__ alpha,
                                                               double *__restrict__ part, double *__restrict__ part2,
                                                               const double *__restrict__ scale,
                                                               const int *__restrict__ done)
{
    __shared__ double sh[kCgThreads];
    const int j = blockIdx.y;
    if (done[j]) return;
    const double a = alpha[j];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRowsPerChunk;
    const int64_t r1 = min(n, r0 + kRowsPerChunk);
    double *xj = X + j * ldx, *rj = R + j * ldw;
    const double *pj = P + j * ldw, *qj = AP + j * ldw;
    double acc = 0.0, acc2 = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kCgThreads) {
        xj[r] = fma(a, pj[r], xj[r]);
        const double rv = fma(-a, qj[r], rj[r]);
        rj[r] = rv;
        acc = fma(rv, rv, acc);
        if (scale) acc2 = fma(rv * scale[r] * scale[r], rv, acc2);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[static_cast<int64_t>(blockIdx.x) * m + j] = t;
    if (scale) {
        __syncthreads();
        const double t2 = block_sum(acc2, sh);
        if (threadIdx.x == 0) part2[static_cast<int64_t>(blockIdx.x) * m + j] = t2;
    }
}

// Per column: the new r^T r, the stop test and beta; one workgroup counts the
// columns still running into ctrl[kRemaining].  With first != 0 the partials
// hold r_0^T r_0 and only rho and the stop test are set.
__global__ __launch_bounds__(kCgThreads) void cg_beta_kernel(const double *__restrict__ part,
                                                             const double *__restrict__ part2, int chunks, int m,
                                                             double *__restrict__ rho, double *__restrict__ beta,
                                                             const double *__restrict__ th2, int *__restrict__ done,
                                                             int *__restrict__ iters, int *__restrict__ ctrl, int first)
{
    __shared__ double sh[kCgThreads];
    double running = 0.0;
    for (int j = threadIdx.x; j < m; j += kCgThreads) {
        if (done[j]) continue;
        const double rr = sum_parts(part, chunks, m, j);
        const double rz = part2 ? sum_parts(part2, chunks, m, j) : rr;  // r^T z (z = M^-1 r)
        if (first) {
            rho[j] = rz;
            iters[j] = 0;
        } else {
            beta[j] = rho[j] > 0.0 ? rz / rho[j] : 0.0;
            rho[j] = rz;
            iters[j] += 1;
        }
        if (rr <= th2[j]) done[j] = 1;
        else running += 1.0;
    }
    const double tot = block_sum(running, sh);
    if (threadIdx.x == 0) ctrl[kRemaining] = static_cast<int>(tot);
}

// p = z + beta p for active columns, z = r or M^-1 r = scale^2 r (grid:
// blocks over rows x m)
__global__ __launch_bounds__(kCgThreads) void cg_p_kernel(double *__restrict__ P, const double *__restrict__ R,
                                                          int64_t ldw, int64_t n, const double *__restrict__ beta,
                                                          const double *__restrict__ scale,
                                                          const int *__restrict__ done, int first)
{
    const int j = blockIdx.y;
    if (done[j] && !first) return;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kCgThreads + threadIdx.x;
    if (r >= n) return;
    const double b = first ? 0.0 : beta[j];
    const double z = scale ? R[j * ldw + r] * scale[r] * scale[r] : R[j * ldw + r];
    P[j * ldw + r] = first ? z : fma(b, P[j * ldw + r], z);
}

// R (ldw) = B (ldb), X = 0, rows < n
__global__ __launch_bounds__(kCgThreads) void cg_init_kernel(const double *__restrict__ B, int64_t ldb,
                                                             double *__restrict__ R, int64_t ldw,
                                                             double *__restrict__ X, int64_t ldx, int64_t n)
{
    const int j = blockIdx.y;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kCgThreads + threadIdx.x;
    if (r >= n) return;
    R[j * ldw + r] = B[j * ldb + r];
    X[j * ldx + r] = 0.0;
}

__global__ void cg_threshold_kernel(const double *__restrict__ part, int chunks, int m, double tol,
                                    double *__restrict__ th2, int *__restrict__ done)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double bb = sum_parts(part, chunks, m, j);
    th2[j] = tol * tol * bb;
    done[j] = 0;
}

}  // namespace

size_t cg_workspace_bytes(int64_t n, int m)
{
    return carve_cg(nullptr, n, m).bytes;
}

bko_status cg_solve(const Operator &op, int m, const double *B, int64_t ldb, double *X, int64_t ldx, double tol,
                    int max_iter, void *work, int *iters_host, bko_solve_info *info, hipStream_t st)
{
    const CgWork w = carve_cg(work, op.n, m);
    const int64_t n = op.n;
    const dim3 rows_grid(static_cast<unsigned>((n + kCgThreads - 1) / kCgThreads), static_cast<unsigned>(m));
    const dim3 chunk_grid(static_cast<unsigned>(w.chunks), static_cast<unsigned>(m));
    const unsigned col_blocks = static_cast<unsigned>((m + 255) / 256);

    // padding rows of P stay zero so the stencil reads defined values
    BKO_HIP(hipGetLastError());
    bko_status rc;
    if ((rc = launch_zero(w.P, sizeof(double) * static_cast<size_t>(w.ldw) * m, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(w.done, sizeof(int) * m, st)) != BKO_OK) return rc;
    hipLaunchKernelGGL(cg_init_kernel, rows_grid, dim3(kCgThreads), 0, st, B, ldb, w.R, w.ldw, X, ldx, n);
    hipLaunchKernelGGL(coldot_kernel, chunk_grid, dim3(kCgThreads), 0, st, w.R, w.ldw, w.R, w.ldw, n, m, w.part,
                       nullptr);
    hipLaunchKernelGGL(cg_threshold_kernel, dim3(col_blocks), dim3(256), 0, st, w.part, w.chunks, m, tol, w.th2,
                       w.done);
    // Jacobi: z = M^-1 r with M^-1 = scale^2
    const double *scale = op.precond == BKO_PRECOND_JACOBI ? op.scale64 : nullptr;
    double *part2 = scale ? w.part2 : nullptr;
    if (scale)
        hipLaunchKernelGGL(coldot_kernel, chunk_grid, dim3(kCgThreads), 0, st, w.R, w.ldw, w.R, w.ldw, n, m, w.part2,
                           nullptr, scale);
    hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kCgThreads), 0, st, w.part, part2, w.chunks, m, w.rho, w.beta,
                       w.th2, w.done, w.iters, w.ctrl, 1);
    hipLaunchKernelGGL(cg_p_kernel, rows_grid, dim3(kCgThreads), 0, st, w.P, w.R, w.ldw, n, w.beta, scale, w.done, 1);
    BKO_HIP(hipGetLastError());

    int remaining = m, launched = 0, chunk = 8;
    while (launched < max_iter) {
        const int todo = std::min(chunk, max_iter - launched);
        for (int it = 0; it < todo; ++it) {
            {
                TimedLaunch tl(kSpmm, st);
                if ((rc = launch_stencil(op, m, w.P, w.ldw, BKO_F64, w.AP, w.ldw, BKO_F64, BKO_F64, nullptr, 0, st)) !=
                    BKO_OK)
                    return rc;
            }
            hipLaunchKernelGGL(coldot_kernel, chunk_grid, dim3(kCgThreads), 0, st, w.P, w.ldw, w.AP, w.ldw, n, m,
                               w.part, w.done);
            hipLaunchKernelGGL(cg_alpha_kernel, dim3(col_blocks), dim3(256), 0, st, w.part, w.chunks, m, w.rho,
                               w.alpha, w.done);
            hipLaunchKernelGGL(cg_update_kernel, chunk_grid, dim3(kCgThreads), 0, st, X, ldx, w.R, w.P, w.AP, w.ldw,
                               n, m, w.alpha, w.part, part2, scale, w.done);
            hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kCgThreads), 0, st, w.part, part2, w.chunks, m, w.rho,
                               w.beta, w.th2, w.done, w.iters, w.ctrl, 0);
            hipLaunchKernelGGL(cg_p_kernel, rows_grid, dim3(kCgThreads), 0, st, w.P, w.R, w.ldw, n, w.beta, scale,
                               w.done, 0);
            BKO_HIP(hipGetLastError());
        }
        launched += todo;
        BKO_HIP(hipMemcpyAsync(&remaining, w.ctrl + kRemaining, sizeof(int), hipMemcpyDeviceToHost, st));
        BKO_HIP(hipStreamSynchronize(st));
        if (remaining == 0) break;
        chunk = std::min(chunk * 2, 128);
    }

    // true FP64 residual of every column: AP = B - A X, then its norms
    if ((rc = launch_stencil(op, m, X, ldx, BKO_F64, w.AP, w.ldw, BKO_F64, BKO_F64, B, ldb, st)) != BKO_OK) return rc;
    std::vector<double> hp(static_cast<size_t>(w.chunks) * m), hb(static_cast<size_t>(w.chunks) * m);
    hipLaunchKernelGGL(coldot_kernel, chunk_grid, dim3(kCgThreads), 0, st, w.AP, w.ldw, w.AP, w.ldw, n, m, w.part,
                       nullptr);
    BKO_HIP(hipMemcpyAsync(hp.data(), w.part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(coldot_kernel, chunk_grid, dim3(kCgThreads), 0, st, B, ldb, B, ldb, n, m, w.part, nullptr);
    BKO_HIP(hipMemcpyAsync(hb.data(), w.part, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st));
    std::vector<int> it(m);
    BKO_HIP(hipMemcpyAsync(it.data(), w.iters, sizeof(int) * m, hipMemcpyDeviceToHost, st));
    BKO_HIP(hipStreamSynchronize(st));
    double worst = 0.0;
    int most = 0;
    for (int j = 0; j < m; ++j) {
        double rr = 0.0, bb = 0.0;
        for (int c = 0; c < w.chunks; ++c) {
            rr += hp[static_cast<size_t>(c) * m + j];
            bb += hb[static_cast<size_t>(c) * m + j];
        }
        const double rel = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? HUGE_VAL : 0.0);
        worst = std::max(worst, rel);
        most = std::max(most, it[j]);
    }
    if (iters_host) std::copy(it.begin(), it.end(), iters_host);
    bko_solve_info inf{};
    inf.iters = most;
    inf.refinements = 0;
    inf.deflated = 0;
    inf.max_rel_res = worst;
    inf.status = remaining == 0 ? BKO_OK : BKO_ENOCONV;
    if (info) *info = inf;
    if (inf.status != BKO_OK) {
        set_error("%d of %d columns did not converge within %d iterations", remaining, m, max_iter);
        return BKO_ENOCONV;
    }
    return BKO_OK;
}

}  // namespace bko
