// Block Krylov solve of A X = B for s right-hand sides sharing one heat
// operator (Sec. III-A, Eq. (4)).
//
// The paper names block CG without fixing a variant.  This is the retooled
// block CG that carries an orthonormal residual basis Q (R = Q C with C
// upper triangular) so that columns converging at different rates do not
// make the s x s systems ill conditioned, with rank-revealing (masked)
// Cholesky factorisations that drop linearly dependent directions instead of
// breaking down.  One iteration, with P the search block:
//     AP    = A P                                   (stencil product)
//     delta = P^T AP          = L_d L_d^T           (FP64 Gram, Cholesky)
//     D    += P delta^+ C                            (solution update)
//     W     = Q - AP delta^+                         (next residual basis)
//     W^T W = L L^T,  S = L^T                        (Cholesky QR)
//     Q     = W S^+,  C = S C,  P = Q + P S^T
// and ||r_j|| = ||C e_j||, so convergence is read off C without a pass.
//
// Storage: the N x s blocks are FP64 or FP32 (compute = BKO_F32); Gram
// matrices, factorisations, the small matrices and the outer residual stay
// FP64.  An outer loop forms R = B - A X in FP64, runs the block iteration
// on A D = R, adds D to X, and stops when max_j ||r_j|| / ||b_j|| <= tol
// (FP64 iterative refinement for the mixed-precision mode).
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 256;
constexpr int kMaxParts = 128;   // Gram partials per product
constexpr int kSmallThreads = 1024;
constexpr int kMaxS = 64;

// --------------------------------------------------------------- layout

struct SmallLayout {
    // doubles
    size_t C, M1, M2, M3, M4, th, total_d;
    // floats (after the doubles)
    size_t M1f, M2f, M3f, M4f, total_f;
};

inline SmallLayout small_layout(int s)
{
    SmallLayout L{};
    const size_t ss = static_cast<size_t>(s) * s;
    size_t o = 0;
    L.C = o; o += ss;
    L.M1 = o; o += ss;
    L.M2 = o; o += ss;
    L.M3 = o; o += ss;
    L.M4 = o; o += ss;
    L.th = o; o += kMaxS;
    L.total_d = align_up(o, 32);
    size_t f = 0;
    L.M1f = f; f += ss;
    L.M2f = f; f += ss;
    L.M3f = f; f += ss;
    L.M4f = f; f += ss;
    L.total_f = align_up(f, 64);
    return L;
}

enum Ctrl { kDone = 0, kIters = 1, kDeflated = 2, kAllDeflated = 3, kNumCtrl = 64 };

struct Workspace {
    int64_t ldw;       // padded rows of every internal block
    double *R64;       // outer residual, FP64
    void *Dv, *Q, *P, *AP, *W;  // inner blocks in the compute storage type
    double *parts;     // Gram partials [kMaxParts][s][s]
    double *smalld;
    float *smallf;
    int *ctrl;
    double *colparts;  // column-norm partials [kMaxParts][s]
    size_t bytes;
};

inline Workspace carve(void *base, int64_t n, int s, bko_dtype compute)
{
    Workspace w{};
    w.ldw = static_cast<int64_t>(align_up(static_cast<size_t>(n), 64));
    const size_t vsz = compute == BKO_F64 ? 8 : 4;
    const size_t blk64 = align_up(sizeof(double) * w.ldw * s, 256);
    const size_t blkv = align_up(vsz * w.ldw * s, 256);
    const SmallLayout SL = small_layout(s);
    char *p = static_cast<char *>(base);
    size_t o = 0;
    w.R64 = reinterpret_cast<double *>(p + o); o += blk64;
    w.Dv = p + o; o += blkv;
    w.Q = p + o; o += blkv;
    w.P = p + o; o += blkv;
    w.AP = p + o; o += blkv;
    w.W = p + o; o += blkv;
    w.parts = reinterpret_cast<double *>(p + o); o += align_up(sizeof(double) * kMaxParts * s * s, 256);
    w.smalld = reinterpret_cast<double *>(p + o); o += align_up(sizeof(double) * SL.total_d, 256);
    w.smallf = reinterpret_cast<float *>(p + o); o += align_up(sizeof(float) * SL.total_f, 256);
    w.ctrl = reinterpret_cast<int *>(p + o); o += 256;
    w.colparts = reinterpret_cast<double *>(p + o); o += align_up(sizeof(double) * kMaxParts * kMaxS, 256);
    w.bytes = o;
    return w;
}

// --------------------------------------------------------------- Gram

// parts[blockIdx.x] = U^T V over the rows owned by this workgroup, in FP64 on
// the FP64 matrix cores.  U, V: ldw x s column-major, rows >= n are zero.
template <class T, int NB, bool kSym>
__global__ __launch_bounds__(kGramThreads) void gram_kernel(const T *__restrict__ U, const T *__restrict__ V,
                                                            int64_t ldw, int s, int64_t rows_per_wg,
                                                            double *__restrict__ parts, const int *__restrict__ ctrl)
{
    if (ctrl && ctrl[kDone]) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15;
    const int lg = lane >> 4;
    const int64_t r_begin = static_cast<int64_t>(blockIdx.x) * rows_per_wg;
    const int64_t r_end = min(ldw, r_begin + rows_per_wg);
    d4 acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    for (int64_t r0 = r_begin + wave * 16; r0 < r_end; r0 += 64) {
        const int64_t row = r0 + lg * 4;
        double u[NB][4], v[NB][4];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int col = b * 16 + li;
            const bool ok = col < s;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                u[b][t] = ok ? static_cast<double>(U[static_cast<int64_t>(col) * ldw + row + t]) : 0.0;
                if constexpr (!kSym) v[b][t] = ok ? static_cast<double>(V[static_cast<int64_t>(col) * ldw + row + t]) : 0.0;
                else v[b][t] = u[b][t];
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(u[a][t], v[b][t], acc[a][b], 0, 0, 0);
    }
    // reduce the four waves through LDS, then write this workgroup's partial
    __shared__ double sh[kMaxS * kMaxS];
    const int ss = s * s;
    for (int e = threadIdx.x; e < ss; e += kGramThreads) sh[e] = 0.0;
    __syncthreads();
    for (int w = 0; w < kGramThreads / 64; ++w) {
        if (wave == w) {
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = a * 16 + mfma_row<true>(lg, r);
                        const int j = b * 16 + li;
                        if (i < s && j < s) sh[i * s + j] += acc[a][b][r];
                    }
        }
        __syncthreads();
    }
    double *out = parts + static_cast<int64_t>(blockIdx.x) * ss;
    for (int e = threadIdx.x; e < ss; e += kGramThreads) out[e] = sh[e];
}

// --------------------------------------------------------------- small dense FP64

// Sum the Gram partials into G (LDS, s x s row-major).
__device__ void reduce_parts(const double *__restrict__ parts, int nparts, int s, double *G)
{
    const int ss = s * s;
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        double acc = 0.0;
        for (int p = 0; p < nparts; ++p) acc += parts[static_cast<int64_t>(p) * ss + e];
        G[e] = acc;
    }
    __syncthreads();
}

// In-place masked Cholesky of the symmetric s x s matrix G (LDS): on return
// the lower triangle holds L with G ~ L L^T on the active index set; a pivot
// below rel_thr * max diag (or not finite) deactivates its index, whose
// column of L is zero.  Returns the number of inactive indices (all threads).
__device__ int masked_cholesky(double *G, int s, double rel_thr, int *active, double *scratch)
{
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int k = 0; k < s; ++k) mx = fmax(mx, G[k * s + k]);
        scratch[0] = mx * rel_thr;
    }
    __syncthreads();
    const double thr = scratch[0];
    for (int k = 0; k < s; ++k) {
        if (threadIdx.x == 0) {
            const double piv = G[k * s + k];
            const bool act = piv > thr && piv > 0.0 && isfinite(piv);
            active[k] = act ? 1 : 0;
            const double lkk = act ? sqrt(piv) : 0.0;
            G[k * s + k] = lkk;
            scratch[1] = act ? 1.0 / lkk : 0.0;
        }
        __syncthreads();
        const double inv = scratch[1];
        for (int i = k + 1 + threadIdx.x; i < s; i += blockDim.x) G[i * s + k] *= inv;
        __syncthreads();
        const int m = s - k - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int i = k + 1 + e / m;
            const int j = k + 1 + e % m;
            if (j <= i) G[i * s + j] -= G[i * s + k] * G[j * s + k];
        }
        __syncthreads();
    }
    // clear the strict upper triangle
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e % s;
        if (j > i) G[e] = 0.0;
    }
    __syncthreads();
    int inactive = 0;
    for (int k = 0; k < s; ++k) inactive += active[k] ? 0 : 1;
    return inactive;
}

// Li = L^+ (inverse on the active set, zero elsewhere), L lower triangular.
__device__ void masked_lower_inverse(const double *L, int s, const int *active, double *Li)
{
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        for (int i = 0; i < s; ++i) {
            double v = 0.0;
            if (i >= j && active[i] && active[j]) {
                v = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) v -= L[i * s + k] * Li[k * s + j];
                v /= L[i * s + i];
            }
            Li[i * s + j] = v;
        }
    }
    __syncthreads();
}

// Store M (row-major s x s in LDS) transposed into global FP64 and FP32:
// out[j * s + k] = M[k][j], the layout the block-update kernels read.
__device__ void store_t(const double *M, int s, double *outd, float *outf)
{
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int j = e / s, k = e % s;
        const double v = M[k * s + j];
        outd[e] = v;
        outf[e] = static_cast<float>(v);
    }
}

// After delta = P^T AP: M1 = delta^+ C (for D += P M1), M2 = delta^+ (for
// W = Q - AP M2).
__global__ __launch_bounds__(kSmallThreads) void small_alpha_kernel(const double *__restrict__ parts, int nparts,
                                                                    int s, double rel_thr, double *smalld,
                                                                    float *smallf, int *ctrl, SmallLayout SL)
{
    if (ctrl[kDone]) return;
    __shared__ double G[kMaxS * kMaxS];
    __shared__ double Li[kMaxS * kMaxS];
    __shared__ int active[kMaxS];
    __shared__ double scratch[4];
    reduce_parts(parts, nparts, s, G);
    masked_cholesky(G, s, rel_thr, active, scratch);
    masked_lower_inverse(G, s, active, Li);
    // E = Li^T Li  (into G: L is no longer needed)
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e % s;
        double acc = 0.0;
        for (int k = max(i, j); k < s; ++k) acc += Li[k * s + i] * Li[k * s + j];
        G[e] = acc;
    }
    __syncthreads();
    store_t(G, s, smalld + SL.M2, smallf + SL.M2f);
    // M1 = E C (C upper triangular), into Li
    const double *C = smalld + SL.C;
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e % s;
        double acc = 0.0;
        for (int k = 0; k <= j; ++k) acc += G[i * s + k] * C[k * s + j];
        Li[e] = acc;
    }
    __syncthreads();
    store_t(Li, s, smalld + SL.M1, smallf + SL.M1f);
}

// After W^T W: L = chol, S = L^T, C <- S C, Q = W S^+ (M3 = S^+), P = Q + P S^T
// (M4 = S^T = L); convergence when ||C e_j|| <= th_j for every column.
// With count == 0 this is the initial QR of the residual (C = I on entry).
__global__ __launch_bounds__(kSmallThreads) void small_beta_kernel(const double *__restrict__ parts, int nparts,
                                                                   int s, double rel_thr, double *smalld,
                                                                   float *smallf, int *ctrl, SmallLayout SL,
                                                                   int count)
{
    if (ctrl[kDone]) return;
    __shared__ double G[kMaxS * kMaxS];
    __shared__ double Li[kMaxS * kMaxS];
    __shared__ int active[kMaxS];
    __shared__ double scratch[4];
    __shared__ int notconv;
    reduce_parts(parts, nparts, s, G);
    const int inactive = masked_cholesky(G, s, rel_thr, active, scratch);
    masked_lower_inverse(G, s, active, Li);
    // M3 = S^+ = Li^T, stored transposed: out[j][k] = M3[k][j] = Li[j][k]
    // M4 = S^T = L,    stored transposed: out[j][k] = M4[k][j] = L[k][j]
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int j = e / s, k = e % s;
        const double v3 = Li[e];
        const double v4 = G[k * s + j];
        smalld[SL.M3 + e] = v3;
        smallf[SL.M3f + e] = static_cast<float>(v3);
        smalld[SL.M4 + e] = v4;
        smallf[SL.M4f + e] = static_cast<float>(v4);
    }
    __syncthreads();
    // Cn = L^T C (both upper triangular), into Li
    double *C = smalld + SL.C;
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e % s;
        double acc = 0.0;
        for (int k = i; k <= j; ++k) acc += G[k * s + i] * C[k * s + j];
        Li[e] = acc;
    }
    if (threadIdx.x == 0) notconv = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        double nrm2 = 0.0;
        for (int i = 0; i <= j; ++i) nrm2 += Li[i * s + j] * Li[i * s + j];
        if (!(sqrt(nrm2) <= smalld[SL.th + j])) atomicAdd(&notconv, 1);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) C[e] = Li[e];
    if (threadIdx.x == 0) {
        ctrl[kIters] += count;
        ctrl[kDeflated] = inactive;
        if (inactive == s) ctrl[kAllDeflated] = 1;
        if (notconv == 0 || inactive == s) ctrl[kDone] = 1;
    }
}

// --------------------------------------------------------------- block updates

// One thread per row; the s x s matrices are read as wave-uniform values.
// D += P M1 ;  W = Q - AP M2
template <class T, int SM>
__global__ __launch_bounds__(256) void update_xw_kernel(int64_t n, int64_t ldw, int s, T *__restrict__ D,
                                                        const T *__restrict__ P, const T *__restrict__ Q,
                                                        const T *__restrict__ AP, T *__restrict__ W,
                                                        const T *__restrict__ M1t, const T *__restrict__ M2t,
                                                        const int *__restrict__ ctrl)
{
    if (ctrl[kDone]) return;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    T p[SM], ap[SM];
#pragma unroll
    for (int k = 0; k < SM; ++k) {
        p[k] = k < s ? P[k * ldw + r] : T(0);
        ap[k] = k < s ? AP[k * ldw + r] : T(0);
    }
    for (int j = 0; j < s; ++j) {
        T a1 = 0, a2 = 0;
#pragma unroll
        for (int k = 0; k < SM; ++k) {
            if (k < s) {
                a1 += p[k] * M1t[j * s + k];
                a2 += ap[k] * M2t[j * s + k];
            }
        }
        D[j * ldw + r] += a1;
        W[j * ldw + r] = Q[j * ldw + r] - a2;
    }
}

// Q = W M3 ; P = Q + P M4   (M3 upper, M4 lower triangular)
template <class T, int SM>
__global__ __launch_bounds__(256) void update_qp_kernel(int64_t n, int64_t ldw, int s, const T *__restrict__ W,
                                                        T *__restrict__ Q, T *__restrict__ P,
                                                        const T *__restrict__ M3t, const T *__restrict__ M4t,
                                                        const int *__restrict__ ctrl)
{
    if (ctrl[kDone]) return;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    T w[SM], p[SM];
#pragma unroll
    for (int k = 0; k < SM; ++k) {
        w[k] = k < s ? W[k * ldw + r] : T(0);
        p[k] = k < s ? P[k * ldw + r] : T(0);
    }
    for (int j = 0; j < s; ++j) {
        T q = 0, pp = 0;
#pragma unroll
        for (int k = 0; k < SM; ++k) {
            if (k < s) {
                if (k <= j) q += w[k] * M3t[j * s + k];
                if (k >= j) pp += p[k] * M4t[j * s + k];
            }
        }
        Q[j * ldw + r] = q;
        P[j * ldw + r] = q + pp;
    }
}

// --------------------------------------------------------------- misc kernels

// colparts[chunk * s + j] = sum over the chunk of column j squared (FP64).
__global__ __launch_bounds__(256) void colnorm_kernel(const double *__restrict__ A, int64_t lda, int64_t n, int s,
                                                      int64_t rows_per_chunk, double *__restrict__ colparts)
{
    const int j = blockIdx.y;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_chunk;
    const int64_t r1 = min(n, r0 + rows_per_chunk);
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const double v = A[j * lda + r];
        acc += v * v;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) colparts[static_cast<int64_t>(blockIdx.x) * s + j] = sh[0];
}

// dst (ldw-padded, type T) = src (FP64, lds)  for rows < n
template <class T>
__global__ __launch_bounds__(256) void cast_in_kernel(const double *__restrict__ src, int64_t lds, T *__restrict__ dst,
                                                      int64_t ldd, int64_t n, int s)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int j = 0; j < s; ++j) dst[j * ldd + r] = static_cast<T>(src[j * lds + r]);
}

// X (FP64) += D (type T)
template <class T>
__global__ __launch_bounds__(256) void add_out_kernel(double *__restrict__ X, int64_t ldx, const T *__restrict__ D,
                                                      int64_t ldd, int64_t n, int s)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int j = 0; j < s; ++j) X[j * ldx + r] += static_cast<double>(D[j * ldd + r]);
}

__global__ void copy_block_kernel(const double *__restrict__ src, int64_t lds, double *__restrict__ dst, int64_t ldd,
                                  int64_t n, int s)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int j = 0; j < s; ++j) dst[j * ldd + r] = src[j * lds + r];
}

__global__ void set_identity_kernel(double *C, int s)
{
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) C[e] = (e / s == e % s) ? 1.0 : 0.0;
}

// --------------------------------------------------------------- driver

template <class T>
struct Inner {
    static constexpr bool kF64 = sizeof(T) == 8;
};

inline int sm_for(int s) { return s <= 8 ? 8 : s <= 16 ? 16 : s <= 32 ? 32 : 64; }

template <class T>
bko_status launch_gram(const T *U, const T *V, int64_t ldw, int s, double *parts, int nparts,
                       const int *ctrl, hipStream_t st)
{
    const int64_t rows = static_cast<int64_t>(align_up(static_cast<size_t>((ldw + nparts - 1) / nparts), 64));
    const int nb = (s + 15) / 16;
    const bool sym = U == V;
    TimedLaunch tl(kGram, st);
#define BKO_GRAM(NB)                                                                                          \
    if (sym) hipLaunchKernelGGL((gram_kernel<T, NB, true>), dim3(nparts), dim3(kGramThreads), 0, st, U, V, ldw, \
                                s, rows, parts, ctrl);                                                        \
    else hipLaunchKernelGGL((gram_kernel<T, NB, false>), dim3(nparts), dim3(kGramThreads), 0, st, U, V, ldw, s, \
                            rows, parts, ctrl);
    if (nb == 1) { BKO_GRAM(1) }
    else if (nb == 2) { BKO_GRAM(2) }
    else if (nb == 3) { BKO_GRAM(3) }
    else { BKO_GRAM(4) }
#undef BKO_GRAM
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class T>
bko_status launch_update_xw(int64_t n, int64_t ldw, int s, T *D, const T *P, const T *Q, const T *AP, T *W,
                            const T *M1t, const T *M2t, const int *ctrl, hipStream_t st)
{
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    TimedLaunch tl(kUpdate, st);
    switch (sm_for(s)) {
    case 8: hipLaunchKernelGGL((update_xw_kernel<T, 8>), dim3(blocks), dim3(256), 0, st, n, ldw, s, D, P, Q, AP, W, M1t, M2t, ctrl); break;
    case 16: hipLaunchKernelGGL((update_xw_kernel<T, 16>), dim3(blocks), dim3(256), 0, st, n, ldw, s, D, P, Q, AP, W, M1t, M2t, ctrl); break;
    case 32: hipLaunchKernelGGL((update_xw_kernel<T, 32>), dim3(blocks), dim3(256), 0, st, n, ldw, s, D, P, Q, AP, W, M1t, M2t, ctrl); break;
    default: hipLaunchKernelGGL((update_xw_kernel<T, 64>), dim3(blocks), dim3(256), 0, st, n, ldw, s, D, P, Q, AP, W, M1t, M2t, ctrl); break;
    }
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class T>
bko_status launch_update_qp(int64_t n, int64_t ldw, int s, const T *W, T *Q, T *P, const T *M3t, const T *M4t,
                            const int *ctrl, hipStream_t st)
{
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    TimedLaunch tl(kUpdate, st);
    switch (sm_for(s)) {
    case 8: hipLaunchKernelGGL((update_qp_kernel<T, 8>), dim3(blocks), dim3(256), 0, st, n, ldw, s, W, Q, P, M3t, M4t, ctrl); break;
    case 16: hipLaunchKernelGGL((update_qp_kernel<T, 16>), dim3(blocks), dim3(256), 0, st, n, ldw, s, W, Q, P, M3t, M4t, ctrl); break;
    case 32: hipLaunchKernelGGL((update_qp_kernel<T, 32>), dim3(blocks), dim3(256), 0, st, n, ldw, s, W, Q, P, M3t, M4t, ctrl); break;
    default: hipLaunchKernelGGL((update_qp_kernel<T, 64>), dim3(blocks), dim3(256), 0, st, n, ldw, s, W, Q, P, M3t, M4t, ctrl); break;
    }
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

// Column norms of an FP64 n x s block, returned on the host.
bko_status host_colnorms(const double *A, int64_t lda, int64_t n, int s, double *colparts, std::vector<double> &out,
                         hipStream_t st)
{
    const int chunks = static_cast<int>(std::min<int64_t>(kMaxParts, (n + 4095) / 4096));
    const int64_t rows = (n + chunks - 1) / chunks;
    hipLaunchKernelGGL(colnorm_kernel, dim3(chunks, s), dim3(256), 0, st, A, lda, n, s, rows, colparts);
    BKO_HIP(hipGetLastError());
    std::vector<double> h(static_cast<size_t>(chunks) * s);
    BKO_HIP(hipMemcpyAsync(h.data(), colparts, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    BKO_HIP(hipStreamSynchronize(st));
    out.assign(s, 0.0);
    for (int c = 0; c < chunks; ++c)
        for (int j = 0; j < s; ++j) out[j] += h[static_cast<size_t>(c) * s + j];
    for (int j = 0; j < s; ++j) out[j] = std::sqrt(out[j]);
    return BKO_OK;
}

// Inner block iteration on A D = R (R = ws.R64, FP64), storage type T.
// th: per-column absolute residual targets.  Returns iterations taken.
template <class T>
bko_status inner_solve(const Operator &op, int s, const Workspace &ws, const std::vector<double> &th, int budget,
                       int &iters_out, int &deflated_out, bool &all_deflated, hipStream_t st)
{
    const int64_t n = op.n, ldw = ws.ldw;
    const SmallLayout SL = small_layout(s);
    const bool f64 = sizeof(T) == 8;
    const double rel_thr = f64 ? 1e-13 : 1e-12;
    const int nparts = static_cast<int>(std::min<int64_t>(kMaxParts, std::max<int64_t>(1, ldw / 1024)));
    T *Dv = static_cast<T *>(ws.Dv), *Q = static_cast<T *>(ws.Q), *P = static_cast<T *>(ws.P);
    T *AP = static_cast<T *>(ws.AP), *W = static_cast<T *>(ws.W);
    const T *M1t = f64 ? reinterpret_cast<const T *>(ws.smalld + SL.M1) : reinterpret_cast<const T *>(ws.smallf + SL.M1f);
    const T *M2t = f64 ? reinterpret_cast<const T *>(ws.smalld + SL.M2) : reinterpret_cast<const T *>(ws.smallf + SL.M2f);
    const T *M3t = f64 ? reinterpret_cast<const T *>(ws.smalld + SL.M3) : reinterpret_cast<const T *>(ws.smallf + SL.M3f);
    const T *M4t = f64 ? reinterpret_cast<const T *>(ws.smalld + SL.M4) : reinterpret_cast<const T *>(ws.smallf + SL.M4f);
    const size_t blkv = sizeof(T) * static_cast<size_t>(ldw) * s;
    bko_status rc;

    // fresh state: blocks zero (padding rows stay zero for the Gram), C = I
    for (void *b : {ws.Dv, ws.Q, ws.P, ws.AP, ws.W})
        if ((rc = launch_zero(b, blkv, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(ws.ctrl, 256, st)) != BKO_OK) return rc;
    hipLaunchKernelGGL(set_identity_kernel, dim3(1), dim3(256), 0, st, ws.smalld + SL.C, s);
    BKO_HIP(hipGetLastError());
    std::vector<double> thp(kMaxS, 0.0);
    std::copy(th.begin(), th.end(), thp.begin());
    BKO_HIP(hipMemcpyAsync(ws.smalld + SL.th, thp.data(), sizeof(double) * kMaxS, hipMemcpyHostToDevice, st));
    const unsigned rblocks = static_cast<unsigned>((n + 255) / 256);
    hipLaunchKernelGGL((cast_in_kernel<T>), dim3(rblocks), dim3(256), 0, st, ws.R64, ldw, W, ldw, n, s);
    BKO_HIP(hipGetLastError());
    // initial QR of the residual: W = Q C
    if ((rc = launch_gram<T>(W, W, ldw, s, ws.parts, nparts, ws.ctrl, st)) != BKO_OK) return rc;
    {
        TimedLaunch tl(kSmall, st);
        hipLaunchKernelGGL(small_beta_kernel, dim3(1), dim3(kSmallThreads), 0, st, ws.parts, nparts, s, rel_thr,
                           ws.smalld, ws.smallf, ws.ctrl, SL, 0);
    }
    BKO_HIP(hipGetLastError());
    if ((rc = launch_update_qp<T>(n, ldw, s, W, Q, P, M3t, M4t, ws.ctrl, st)) != BKO_OK) return rc;

    const bko_dtype vt = f64 ? BKO_F64 : BKO_F32;
    int h_ctrl[4] = {0, 0, 0, 0};
    int launched = 0;
    int chunk = 4;
    while (true) {
        const int todo = std::min(chunk, budget - launched);
        for (int it = 0; it < todo; ++it) {
            {
                TimedLaunch tl(kSpmm, st);
                if ((rc = launch_stencil(op, s, P, ldw, vt, AP, ldw, vt, vt, nullptr, 0, st, ws.ctrl)) != BKO_OK)
                    return rc;
            }
            if ((rc = launch_gram<T>(P, AP, ldw, s, ws.parts, nparts, ws.ctrl, st)) != BKO_OK) return rc;
            {
                TimedLaunch tl(kSmall, st);
                hipLaunchKernelGGL(small_alpha_kernel, dim3(1), dim3(kSmallThreads), 0, st, ws.parts, nparts, s,
                                   rel_thr, ws.smalld, ws.smallf, ws.ctrl, SL);
            }
            BKO_HIP(hipGetLastError());
            if ((rc = launch_update_xw<T>(n, ldw, s, Dv, P, Q, AP, W, M1t, M2t, ws.ctrl, st)) != BKO_OK) return rc;
            if ((rc = launch_gram<T>(W, W, ldw, s, ws.parts, nparts, ws.ctrl, st)) != BKO_OK) return rc;
            {
                TimedLaunch tl(kSmall, st);
                hipLaunchKernelGGL(small_beta_kernel, dim3(1), dim3(kSmallThreads), 0, st, ws.parts, nparts, s,
                                   rel_thr, ws.smalld, ws.smallf, ws.ctrl, SL, 1);
            }
            BKO_HIP(hipGetLastError());
            if ((rc = launch_update_qp<T>(n, ldw, s, W, Q, P, M3t, M4t, ws.ctrl, st)) != BKO_OK) return rc;
        }
        launched += todo;
        BKO_HIP(hipMemcpyAsync(h_ctrl, ws.ctrl, sizeof(h_ctrl), hipMemcpyDeviceToHost, st));
        BKO_HIP(hipStreamSynchronize(st));
        if (h_ctrl[kDone] || launched >= budget) break;
        chunk = std::min(chunk * 2, 32);
    }
    iters_out = h_ctrl[kIters];
    deflated_out = h_ctrl[kDeflated];
    all_deflated = h_ctrl[kAllDeflated] != 0;
    // X += D happens in the caller
    return BKO_OK;
}

}  // namespace

size_t solve_workspace_bytes(int64_t n, int s, bko_dtype compute)
{
    return carve(nullptr, n, s, compute).bytes;
}

bko_status block_solve(const Operator &op, int s, const double *B, int64_t ldb, double *X, int64_t ldx,
                       const double *X0, int64_t ldx0, bko_dtype compute, double tol, int max_iter, void *work,
                       size_t work_bytes, bko_solve_info *info, hipStream_t st)
{
    (void)work_bytes;
    const Workspace ws = carve(work, op.n, s, compute);
    const int64_t n = op.n;
    const unsigned rblocks = static_cast<unsigned>((n + 255) / 256);
    bko_status rc;
    std::vector<double> bnorm, rnorm;
    if ((rc = host_colnorms(B, ldb, n, s, ws.colparts, bnorm, st)) != BKO_OK) return rc;
    for (int j = 0; j < s; ++j)
        if (!std::isfinite(bnorm[j])) {
            set_error("right-hand side column %d is not finite", j);
            return BKO_EINVAL;
        }
    // X = X0 or 0
    if (X0 == nullptr) {
        for (int j = 0; j < s; ++j)
            if ((rc = launch_zero(X + j * ldx, sizeof(double) * n, st)) != BKO_OK) return rc;
    } else if (X0 != X) {
        hipLaunchKernelGGL(copy_block_kernel, dim3(rblocks), dim3(256), 0, st, X0, ldx0, X, ldx, n, s);
        BKO_HIP(hipGetLastError());
    }
    bko_solve_info inf{};
    inf.status = BKO_ENOCONV;
    double prev_rel = HUGE_VAL;
    int stagnant = 0;
    const double inner_rel_f32 = 1e-5;
    for (int outer = 0; outer < 100; ++outer) {
        // R = B - A X in FP64 (padding rows of R64 stay untouched; the cast
        // below only reads rows < n)
        {
            TimedLaunch tl(kResid, st);
            if ((rc = launch_stencil(op, s, X, ldx, BKO_F64, ws.R64, ws.ldw, BKO_F64, BKO_F64, B, ldb, st)) != BKO_OK)
                return rc;
        }
        if ((rc = host_colnorms(ws.R64, ws.ldw, n, s, ws.colparts, rnorm, st)) != BKO_OK) return rc;
        double rel = 0.0;
        bool finite = true;
        for (int j = 0; j < s; ++j) {
            finite = finite && std::isfinite(rnorm[j]);
            rel = std::max(rel, bnorm[j] > 0 ? rnorm[j] / bnorm[j] : (rnorm[j] > 0 ? HUGE_VAL : 0.0));
        }
        inf.max_rel_res = rel;
        if (!finite) {
            set_error("residual is not finite (initial guess or operator invalid)");
            inf.status = BKO_EINVAL;
            break;
        }
        if (rel <= tol) {
            inf.status = BKO_OK;
            break;
        }
        if (inf.iters >= max_iter) {
            inf.status = BKO_ENOCONV;
            break;
        }
        if (rel > 0.5 * prev_rel) {
            if (++stagnant >= 3) {
                inf.status = BKO_EBREAKDOWN;
                break;
            }
        } else {
            stagnant = 0;
        }
        prev_rel = rel;
        std::vector<double> th(s);
        for (int j = 0; j < s; ++j) {
            const double target = 0.5 * tol * bnorm[j];
            th[j] = compute == BKO_F64 ? target : std::max(target, inner_rel_f32 * rnorm[j]);
        }
        int it = 0, defl = 0;
        bool alldefl = false;
        const int budget = max_iter - inf.iters;
        if (compute == BKO_F64) rc = inner_solve<double>(op, s, ws, th, budget, it, defl, alldefl, st);
        else rc = inner_solve<float>(op, s, ws, th, budget, it, defl, alldefl, st);
        if (rc != BKO_OK) return rc;
        inf.iters += it;
        inf.refinements += 1;
        inf.deflated = std::max(inf.deflated, defl);
        if (compute == BKO_F64)
            hipLaunchKernelGGL((add_out_kernel<double>), dim3(rblocks), dim3(256), 0, st, X, ldx,
                               static_cast<const double *>(ws.Dv), ws.ldw, n, s);
        else
            hipLaunchKernelGGL((add_out_kernel<float>), dim3(rblocks), dim3(256), 0, st, X, ldx,
                               static_cast<const float *>(ws.Dv), ws.ldw, n, s);
        BKO_HIP(hipGetLastError());
    }
    BKO_HIP(hipStreamSynchronize(st));
    if (info) *info = inf;
    if (inf.status == BKO_ENOCONV) set_error("no convergence within %d iterations (rel res %.3e)", max_iter, inf.max_rel_res);
    if (inf.status == BKO_EBREAKDOWN) set_error("block iteration stagnated at rel res %.3e", inf.max_rel_res);
    return static_cast<bko_status>(inf.status);
}

}  // namespace bko
