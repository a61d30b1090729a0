// Block Krylov solve of A X = B for s right-hand sides sharing one heat
// operator (Sec. III-A, Eq. (4)).
//
// The paper names block CG without fixing a variant.  This is the retooled
// block CG that carries an orthonormal residual basis Q (R = Q C) so that
// columns converging at different rates do not make the s x s systems ill
// conditioned, with rank-revealing factorisations that drop linearly
// dependent directions instead of breaking down.  One iteration, with P the
// search block:
//     AP    = A P                                  (stencil product)
//     delta = P^T AP                               (FP64 Gram)
//     W     = Q - AP delta^+                       (next residual basis)
//     W^T W = S^T S  (S upper triangular)          (Cholesky QR, FP64)
//     D    += P delta^+ C ;  Q = W S^+ ;  P = Q + P S^T ;  C = S C
// and ||r_j|| = ||C e_j||, so convergence is read off C without a pass over
// the residual.
//
// Kernels per iteration, all on one stream with no host round trip; the
// kernel boundary is the only grid-wide synchronisation (an in-kernel fence
// per workgroup costs far more on this chip than the boundary):
//   spmm        AP = A P                       (stencil.hip)
//   gram        per-workgroup P^T AP partials on the FP64 matrix cores
//   reduce      the partials summed entry by entry, in index order
//   factor      one 1024-thread workgroup: delta^+ and delta^+ C
//   update_w    W = Q - AP delta^+ on the matrix cores, and the W^T W
//               partials from the same registers (the 16x16 result layout is
//               the operand layout of the FP64 Gram product)
//   reduce
//   factor      W^T W = S^T S, C <- S C, convergence test
//   update_dqp  D += P delta^+ C, Q = W S^+, P = Q + P S^T
//
// The s x s factorisations are an LDL^T elimination of [G | I] without
// pivoting in which a pivot below a relative threshold deactivates its index
// (its row and column of every derived matrix are zero): one barrier per
// pivot, every thread owning fixed entries.
//
// Storage: the N x s blocks are FP64 or FP32 (compute = BKO_F32); Gram
// matrices, factorisations, small matrices and the outer residual are FP64.
// An outer loop forms R = B - A X in FP64, runs the block iteration on
// A D = R, adds D to X, and stops when max_j ||r_j|| / ||b_j|| <= tol (FP64
// iterative refinement in the mixed-precision mode).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;      // block kernels
constexpr int kFacThreads = 256;   // factorisation kernel
constexpr int kMaxS = 64;
constexpr int kMaxBlocks = 512;    // partial producers per launch
constexpr int kRedBlocks = 64;     // reducer workgroups
constexpr int kTileRows = 256;     // rows per workgroup tile (4 waves x 64)

// ------------------------------------------------------------------ layout

enum Ctrl { kConverged = 0, kStop = 1, kIters = 2, kDeflated = 3, kAllDeflated = 4 };

struct Small {
    // FP64, row-major s x s: M[k][j] maps input column k to output column j
    double *C, *M1, *M2, *M3, *M4, *th;
    // FP32 copies for the FP32 block kernels
    float *M1f, *M2f, *M3f, *M4f;
};

struct Workspace {
    int64_t ldw;                 // padded rows of every internal block
    double *R64;                 // outer residual, FP64
    void *Dv, *Q, *P, *AP, *W;   // inner blocks in the storage type
    Small sm;
    double *parts;               // Gram partials [kMaxBlocks][s][s]
    double *gram;                // reduced Gram [s][s]
    int *ctrl;
    double *colparts;            // column-norm partials [128][s]
    size_t bytes;
};

inline Workspace carve(void *base, int64_t n, int s, bko_dtype compute)
{
    Workspace w{};
    w.ldw = static_cast<int64_t>(align_up(static_cast<size_t>(n), kTileRows));
    const size_t vsz = compute == BKO_F64 ? 8 : 4;
    const size_t ss = static_cast<size_t>(s) * s;
    char *p = static_cast<char *>(base);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *q = p + o;
        o = align_up(o + bytes, 256);
        return q;
    };
    w.R64 = reinterpret_cast<double *>(take(sizeof(double) * w.ldw * s));
    w.Dv = take(vsz * w.ldw * s);
    w.Q = take(vsz * w.ldw * s);
    w.P = take(vsz * w.ldw * s);
    w.AP = take(vsz * w.ldw * s);
    w.W = take(vsz * w.ldw * s);
    w.sm.C = reinterpret_cast<double *>(take(sizeof(double) * ss));
    w.sm.M1 = reinterpret_cast<double *>(take(sizeof(double) * ss));
    w.sm.M2 = reinterpret_cast<double *>(take(sizeof(double) * ss));
    w.sm.M3 = reinterpret_cast<double *>(take(sizeof(double) * ss));
    w.sm.M4 = reinterpret_cast<double *>(take(sizeof(double) * ss));
    w.sm.th = reinterpret_cast<double *>(take(sizeof(double) * kMaxS));
    w.sm.M1f = reinterpret_cast<float *>(take(sizeof(float) * ss));
    w.sm.M2f = reinterpret_cast<float *>(take(sizeof(float) * ss));
    w.sm.M3f = reinterpret_cast<float *>(take(sizeof(float) * ss));
    w.sm.M4f = reinterpret_cast<float *>(take(sizeof(float) * ss));
    w.parts = reinterpret_cast<double *>(take(sizeof(double) * ss * kMaxBlocks));
    w.gram = reinterpret_cast<double *>(take(sizeof(double) * ss));
    w.ctrl = reinterpret_cast<int *>(take(sizeof(int) * 64));
    w.colparts = reinterpret_cast<double *>(take(sizeof(double) * 128 * kMaxS));
    w.bytes = o;
    return w;
}

// ------------------------------------------------------------------ matrix-core helpers

template <class T> struct MF;
template <> struct MF<float> {
    using V = f4;
    static constexpr bool kF64 = false;
    __device__ static inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct MF<double> {
    using V = d4;
    static constexpr bool kF64 = true;
    __device__ static inline V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

__device__ inline d4 mma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// index of the (a, b) upper block, a <= b < NB
template <int NB> __device__ constexpr int ublock(int a, int b) { return a * NB - a * (a - 1) / 2 + (b - a); }

// ------------------------------------------------------------------ Gram partials

// Sum the four waves' 16x16 FP64 blocks into an s x s partial in LDS and
// write it to parts[blockIdx.x].  kSym: only upper blocks were formed.
template <int NB, bool kSym, int NBLK>
__device__ void publish_partial(const d4 (&g)[NBLK], int s, double *lds, double *parts)
{
    const int ss = s * s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    for (int e = threadIdx.x; e < ss; e += kThreads) lds[e] = 0.0;
    __syncthreads();
    for (int wv = 0; wv < kThreads / 64; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = kSym ? a : 0; b < NB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = a * 16 + mfma_row<true>(lg, r), j = b * 16 + li;
                        if (i < s && j < s) {
                            const double v = kSym ? g[ublock<NB>(a, b)][r] : g[a * NB + b][r];
                            lds[i * s + j] += v;
                            if (kSym && a != b) lds[j * s + i] += v;
                        }
                    }
        }
        __syncthreads();
    }
    double *out = parts + static_cast<size_t>(blockIdx.x) * ss;
    for (int e = threadIdx.x; e < ss; e += kThreads) out[e] = lds[e];
}

// P^T AP over this workgroup's row tiles.
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void gram_kernel(const T *__restrict__ P, const T *__restrict__ AP, int64_t ldw,
                                                        int s, double *__restrict__ parts, const int *__restrict__ ctrl)
{
    if (ctrl[kConverged]) return;
    __shared__ double lds[kMaxS * kMaxS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t ntiles = ldw / kTileRows;
    d4 acc[NB * NB];
#pragma unroll
    for (int q = 0; q < NB * NB; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int rb = 0; rb < 4; ++rb) {
            // rows row + t feed MFMA step t for lane group lg: any bijection of
            // rows onto k slots works, since the product sums over rows
            const int64_t row = tile * kTileRows + wave * 64 + rb * 16 + lg * 4;
            double u[NB][4], v[NB][4];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int col = b * 16 + li;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    u[b][t] = col < s ? static_cast<double>(P[col * ldw + row + t]) : 0.0;
                    v[b][t] = col < s ? static_cast<double>(AP[col * ldw + row + t]) : 0.0;
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[a * NB + b] = mma64(u[a][t], v[b][t], acc[a * NB + b]);
        }
    }
    publish_partial<NB, false>(acc, s, lds, parts);
}

// gram = sum over p < nparts of parts[p], entry by entry in index order.
__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(const double *__restrict__ parts, int nparts, int ss,
                                                               double *__restrict__ gram, const int *__restrict__ ctrl)
{
    if (ctrl[kConverged]) return;
    __shared__ double sh[kThreads];
    const int per = (ss + gridDim.x - 1) / gridDim.x;  // entries of this workgroup (<= 64)
    const int slices = kThreads / per;
    const int tid = threadIdx.x;
    const int le = tid % per, sl = tid / per;
    const int e = blockIdx.x * per + le;
    double a = 0.0;
    if (sl < slices && e < ss) {
        // slice sl sums partials sl, sl + slices, ... ; 8 loads in flight
        for (int p0 = sl; p0 < nparts; p0 += 8 * slices) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = p0 + q * slices;
                v[q] = p < nparts ? parts[static_cast<size_t>(p) * ss + e] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) a += v[q];
        }
    }
    sh[tid] = a;
    __syncthreads();
    if (sl == 0 && e < ss) {
        double tot = 0.0;
        for (int q = 0; q < slices; ++q) tot += sh[q * per + le];
        gram[e] = tot;
    }
}

// ------------------------------------------------------------------ factorisation (one workgroup)

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Masked LDL^T elimination of [G | I] by one wavefront, for s <= SP <= 32:
// lane c holds column c of the 2 SP columns in registers; each pivot row of
// the column is broadcast with readlane, so no LDS traffic or barrier per
// pivot.  Indices s <= i < SP are decoupled padding with pivot gmax.
// Writes the result (A[i][j], j < 2s: left half U, right half E) to LDS.
template <int SP>
__device__ __forceinline__ void wave_eliminate(const double *__restrict__ gram, int s, double rel_thr, double *A,
                                               int *active)
{
    const int lane = threadIdx.x & 63;
    const int w = 2 * s;
    double gmax = lane < s ? gram[lane * s + lane] : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off));
    const double thr = rel_thr * gmax;
    double a[SP];
#pragma unroll
    for (int i = 0; i < SP; ++i) {
        if (lane < SP)
            a[i] = (i < s && lane < s) ? 0.5 * (gram[i * s + lane] + gram[lane * s + i]) : (i == lane ? gmax : 0.0);
        else
            a[i] = (i == lane - SP) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int k = 0; k < SP; ++k) {
        const double p = readlane_f64(a[k], k);
        const bool act = p > thr && isfinite(p);
        // this column's pivot-row entry, scaled; zero when the pivot is inactive
        const double m = act ? -a[k] * (1.0 / p) : 0.0;
#pragma unroll
        for (int i = k + 1; i < SP; ++i) a[i] = fma(readlane_f64(a[i], k), m, a[i]);
        if (lane == 0 && k < s) active[k] = act ? 1 : 0;
    }
    const int col = lane < SP ? (lane < s ? lane : -1) : (lane - SP < s ? s + lane - SP : -1);
    if (lane < 2 * SP && col >= 0) {
#pragma unroll
        for (int i = 0; i < SP; ++i)
            if (i < s) A[i * w + col] = a[i];
    }
}

// Publish pivot row r of the register-held [G | I], its reciprocal pivot
// (*inv) and column r into the LDS vectors rn / cn.
template <int E>
__device__ __forceinline__ void publish_pivot(const double (&a)[E], int i, int j0, int w, bool live, int r, double *rn,
                                              double *cn, double *inv)
{
    if (!live) return;
    if (i == r) {
#pragma unroll
        for (int q = 0; q < E; ++q)
            if (j0 + q < w) rn[j0 + q] = a[q];
    }
#pragma unroll
    for (int q = 0; q < E; ++q) {
        if (j0 + q == r) {
            cn[i] = a[q];
            if (i == r) *inv = 1.0 / a[q];  // read only when the pivot is active
        }
    }
}

// Factor the reduced Gram.  mode 0: delta -> M2 = delta^+, M1 = delta^+ C.
// mode 1 / 2: W^T W -> S = D^{1/2} Lunit^T, Linv = D^{-1/2} E; C <- S C;
// M3[k][j] = Linv[j][k] (Q = W S^+), M4[k][j] = S[j][k] (P = Q + P S^T);
// converged when ||C e_j|| <= th_j for every column (mode 2 is the first QR
// of the residual and is not counted as an iteration).
//
// Work layout: each of the 256 threads owns E consecutive entries of one row
// of [G | I] in registers; per pivot the owners publish the pivot row (with
// its reciprocal) and column into double-buffered LDS vectors, one barrier
// per pivot.  The s x s products afterwards use the same row-segment
// ownership with E / 2 outputs per thread.
// SP > 0 selects the one-wavefront elimination (s <= SP <= 32).
template <int E, int SP>
__global__ __launch_bounds__(kFacThreads) void factor_kernel(const double *__restrict__ gram, int s, double rel_thr,
                                                             Small sm, int *ctrl, int mode)
{
    if (ctrl[kConverged]) return;
    constexpr int E2 = E > 1 ? E / 2 : 1;
    constexpr int EA = SP > 0 ? 1 : E;  // register row segment of the LDS elimination
    extern __shared__ __align__(16) double lds[];
    const int ss = s * s, w = 2 * s;
    // every region is padded by E doubles so that a row segment can be read
    // whole; padding is zeroed, masked lanes multiply it by zero
    double *A = lds;                        // s x 2s
    double *G = A + 2 * ss + E;             // s x s scratch
    double *Cl = G + ss + E;                // C
    double *rowbuf = Cl + ss + E;           // 2 x (w + E)
    double *colbuf = rowbuf + 2 * (w + E);  // 2 x s
    __shared__ int active[kMaxS];
    __shared__ double dv[kMaxS];
    __shared__ double invb[2];
    __shared__ double gmax;
    __shared__ int notconv;
    const int tid = threadIdx.x;
    for (int e = tid; e < E; e += kFacThreads) {
        A[2 * ss + e] = 0.0;
        G[ss + e] = 0.0;
        Cl[ss + e] = 0.0;
        rowbuf[w + e] = 0.0;
        rowbuf[2 * w + E + e] = 0.0;
    }
    for (int e = tid; e < ss; e += kFacThreads) Cl[e] = sm.C[e];
    if (tid == 0) notconv = 0;
    if constexpr (SP > 0) {
        if (tid < 64) wave_eliminate<SP>(gram, s, rel_thr, A, active);
    } else {
        const int tpr = (w + EA - 1) / EA;
        const int i = tid / tpr, j0 = (tid % tpr) * EA;
        const bool live = i < s;
        double a[EA];
#pragma unroll
        for (int q = 0; q < EA; ++q) {
            const int j = j0 + q;
            a[q] = 0.0;
            if (live && j < w) a[q] = j < s ? 0.5 * (gram[i * s + j] + gram[j * s + i]) : (j - s == i ? 1.0 : 0.0);
        }
        if (tid < 64) {
            double v = tid < s ? gram[tid * s + tid] : 0.0;
            for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
            if (tid == 0) gmax = v;
        }
        publish_pivot<EA>(a, i, j0, w, live, 0, rowbuf, colbuf, &invb[0]);
        __syncthreads();
        const double thr = rel_thr * gmax;
        const int ic = live ? i : 0;
        for (int k = 0; k < s; ++k) {
            const int b = k & 1;
            const double *rb = rowbuf + b * (w + E);
            const double *cb = colbuf + b * s;
            const double p = rb[k];
            const bool act = p > thr && isfinite(p);
            // branch-free update: read the whole pivot-row segment, mask the multiplier
            double r[EA];
#pragma unroll
            for (int q = 0; q < EA; ++q) r[q] = rb[j0 + q];
            const double cv = cb[ic];
            const double l = (act && live && i > k) ? cv * invb[b] : 0.0;
#pragma unroll
            for (int q = 0; q < EA; ++q) {
                const int j = j0 + q;
                const bool upd = (j > k && j < s) || (j >= s && j <= s + k);
                a[q] = fma(upd ? -l : 0.0, r[q], a[q]);
            }
            if (k + 1 < s)
                publish_pivot<EA>(a, i, j0, w, live, k + 1, rowbuf + (b ^ 1) * (w + E), colbuf + (b ^ 1) * s,
                                  &invb[b ^ 1]);
            if (tid == 0) active[k] = act ? 1 : 0;
            __syncthreads();
        }
        if (live) {
#pragma unroll
            for (int q = 0; q < EA; ++q)
                if (j0 + q < w) A[i * w + j0 + q] = a[q];
        }
    }
    __syncthreads();
    for (int k = tid; k < s; k += kFacThreads)
        dv[k] = !active[k] ? 0.0 : (mode == 0 ? 1.0 / A[k * w + k] : 1.0 / sqrt(A[k * w + k]));
    __syncthreads();
    int inactive = 0;
    for (int k = 0; k < s; ++k) inactive += active[k] ? 0 : 1;
    // s x s outputs: thread owns row i2, columns j2 .. j2 + E2
    const int tpr2 = (s + E2 - 1) / E2;
    const int i2 = tid / tpr2, j2 = (tid % tpr2) * E2;
    const bool live2 = i2 < s;
    double acc[E2];
    if (mode == 0) {
        // delta^+[i][j] = sum_{k >= max(i,j)} E[k][i] E[k][j] / d_k, E = right half
#pragma unroll
        for (int q = 0; q < E2; ++q) acc[q] = 0.0;
        if (live2) {
            for (int k = i2; k < s; ++k) {
                const double c = A[k * w + s + i2] * dv[k];
#pragma unroll
                for (int q = 0; q < E2; ++q)
                    acc[q] += c * A[k * w + s + j2 + q];  // columns >= s: padding, not stored
            }
#pragma unroll
            for (int q = 0; q < E2; ++q) {
                if (j2 + q < s) {
                    const int e = i2 * s + j2 + q;
                    G[e] = acc[q];
                    sm.M2[e] = acc[q];
                    sm.M2f[e] = static_cast<float>(acc[q]);
                }
            }
        }
        __syncthreads();
        // M1 = delta^+ C
#pragma unroll
        for (int q = 0; q < E2; ++q) acc[q] = 0.0;
        if (live2) {
            for (int k = 0; k < s; ++k) {
                const double c = G[i2 * s + k];
#pragma unroll
                for (int q = 0; q < E2; ++q)
                    acc[q] += c * Cl[k * s + j2 + q];
            }
#pragma unroll
            for (int q = 0; q < E2; ++q) {
                if (j2 + q < s) {
                    const int e = i2 * s + j2 + q;
                    sm.M1[e] = acc[q];
                    sm.M1f[e] = static_cast<float>(acc[q]);
                }
            }
        }
        return;
    }
    // S[i][k] = U[i][k] dv[i] (k >= i);  Cn = S C into G
#pragma unroll
    for (int q = 0; q < E2; ++q) acc[q] = 0.0;
    if (live2) {
        for (int k = i2; k < s; ++k) {
            const double c = A[i2 * w + k];
#pragma unroll
            for (int q = 0; q < E2; ++q)
                acc[q] += c * Cl[k * s + j2 + q];
        }
#pragma unroll
        for (int q = 0; q < E2; ++q)
            if (j2 + q < s) G[i2 * s + j2 + q] = acc[q] * dv[i2];
    }
    // M3[k][j] = Linv[j][k] = E[j][k] dv[j] (k <= j);  M4[k][j] = S[j][k] = U[j][k] dv[j] (k >= j)
    for (int e = tid; e < ss; e += kFacThreads) {
        const int k = e / s, j = e % s;
        const double m3 = k <= j ? A[j * w + s + k] * dv[j] : 0.0;
        const double m4 = k >= j ? A[j * w + k] * dv[j] : 0.0;
        sm.M3[e] = m3;
        sm.M3f[e] = static_cast<float>(m3);
        sm.M4[e] = m4;
        sm.M4f[e] = static_cast<float>(m4);
    }
    __syncthreads();
    for (int j = tid; j < s; j += kFacThreads) {
        double n0 = 0.0, n1 = 0.0;
        int r = 0;
        for (; r + 1 <= j; r += 2) {
            n0 += G[r * s + j] * G[r * s + j];
            n1 += G[(r + 1) * s + j] * G[(r + 1) * s + j];
        }
        if (r <= j) n0 += G[r * s + j] * G[r * s + j];
        if (!(sqrt(n0 + n1) <= sm.th[j])) atomicAdd(&notconv, 1);
    }
    for (int e = tid; e < ss; e += kFacThreads) sm.C[e] = G[e];
    __syncthreads();
    if (tid == 0) {
        ctrl[kIters] += mode == 1 ? 1 : 0;
        ctrl[kDeflated] = inactive;
        if (inactive == s) ctrl[kAllDeflated] = 1;
        if (notconv == 0 || inactive == s) ctrl[kConverged] = 1;
    }
}

// Smallest row-segment width E (power of two) with s rows x ceil(2s / E)
// threads fitting one workgroup.
inline int factor_segment(int s)
{
    int e = 1;
    while (s * ((2 * s + e - 1) / e) > kFacThreads) e *= 2;
    return e;
}

// ------------------------------------------------------------------ block updates

// W = Q - AP M2 (matrix cores in the storage precision) and the W^T W
// partials from the same registers.  With init != 0, W already holds the
// residual and only its Gram is formed.
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void update_w_kernel(const T *__restrict__ Q, const T *__restrict__ AP,
                                                            T *__restrict__ W, const T *__restrict__ M2g, int64_t ldw,
                                                            int s, double *__restrict__ parts, const int *__restrict__ ctrl,
                                                            int init)
{
    if (ctrl[kConverged]) return;
    using V = typename MF<T>::V;
    constexpr bool kF64 = MF<T>::kF64;
    constexpr int KS = 4 * NB;  // k steps of 4 over the padded width 16 NB
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    __shared__ T Ms[SP * MST];  // -M2
    __shared__ double lds[kMaxS * kMaxS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    if (!init) {
        for (int e = threadIdx.x; e < SP * MST; e += kThreads) {
            const int k = e / MST, j = e % MST;
            Ms[e] = (k < s && j < s) ? -M2g[k * s + j] : T(0);
        }
        __syncthreads();
    }
    d4 g[NB * (NB + 1) / 2];
#pragma unroll
    for (int q = 0; q < NB * (NB + 1) / 2; ++q) g[q] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t ntiles = ldw / kTileRows;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t r0 = tile * kTileRows + wave * 64 + rb * 16;
            T a[KS];
            if (!init) {
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const int col = 4 * t + lg;
                    a[t] = col < s ? AP[col * ldw + r0 + li] : T(0);
                }
            }
            V wv[NB];
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int colj = jb * 16 + li;
                V acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = r0 + mfma_row<kF64>(lg, r);
                    acc[r] = colj < s ? (init ? W[colj * ldw + row] : Q[colj * ldw + row]) : T(0);
                }
                if (!init) {
#pragma unroll
                    for (int t = 0; t < KS; ++t) acc = MF<T>::mma(a[t], Ms[(4 * t + lg) * MST + colj], acc);
                    if (colj < s) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) W[colj * ldw + r0 + mfma_row<kF64>(lg, r)] = acc[r];
                    }
                }
                wv[jb] = acc;
            }
            // W^T W: result register r of lane group lg holds row
            // mfma_row(lg, r) of the block -- the k slot lg of an FP64 step
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int ab = 0; ab < NB; ++ab)
#pragma unroll
                    for (int bb = ab; bb < NB; ++bb)
                        g[ublock<NB>(ab, bb)] = mma64(static_cast<double>(wv[ab][r]), static_cast<double>(wv[bb][r]),
                                                      g[ublock<NB>(ab, bb)]);
        }
    }
    publish_partial<NB, true>(g, s, lds, parts);
}

// D += P M1 ;  Q = W M3 ;  P = Q + P M4   (matrix cores, storage precision)
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void update_dqp_kernel(T *__restrict__ D, T *__restrict__ P, T *__restrict__ Q,
                                                              const T *__restrict__ W, const T *__restrict__ M1g,
                                                              const T *__restrict__ M3g, const T *__restrict__ M4g,
                                                              int64_t ldw, int s, const int *__restrict__ ctrl)
{
    if (ctrl[kStop]) return;
    using V = typename MF<T>::V;
    constexpr bool kF64 = MF<T>::kF64;
    constexpr int KS = 4 * NB;
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    extern __shared__ __align__(16) double lds[];
    T *M1 = reinterpret_cast<T *>(lds);
    T *M3 = M1 + SP * MST;
    T *M4 = M3 + SP * MST;
    for (int e = threadIdx.x; e < SP * MST; e += kThreads) {
        const int k = e / MST, j = e % MST;
        const bool ok = k < s && j < s;
        M1[e] = ok ? M1g[k * s + j] : T(0);
        M3[e] = ok ? M3g[k * s + j] : T(0);
        M4[e] = ok ? M4g[k * s + j] : T(0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t ntiles = ldw / kTileRows;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t r0 = tile * kTileRows + wave * 64 + rb * 16;
            T pa[KS], wa[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int col = 4 * t + lg;
                pa[t] = col < s ? P[col * ldw + r0 + li] : T(0);
                wa[t] = col < s ? W[col * ldw + r0 + li] : T(0);
            }
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int colj = jb * 16 + li;
                V ad, aq;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ad[r] = colj < s ? D[colj * ldw + r0 + mfma_row<kF64>(lg, r)] : T(0);
                    aq[r] = T(0);
                }
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const int k = 4 * t + lg;
                    ad = MF<T>::mma(pa[t], M1[k * MST + colj], ad);
                    aq = MF<T>::mma(wa[t], M3[k * MST + colj], aq);
                }
                V ap = aq;
#pragma unroll
                for (int t = 0; t < KS; ++t) ap = MF<T>::mma(pa[t], M4[(4 * t + lg) * MST + colj], ap);
                if (colj < s) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t idx = colj * ldw + r0 + mfma_row<kF64>(lg, r);
                        D[idx] = ad[r];
                        Q[idx] = aq[r];
                        P[idx] = ap[r];
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ misc kernels

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

// ------------------------------------------------------------------ host side

inline int nb_for(int s) { return (s + 15) / 16; }

inline unsigned grid_for(int64_t ldw)
{
    return static_cast<unsigned>(std::min<int64_t>(ldw / kTileRows, kMaxBlocks));
}

enum Step { kStepGram = 0, kStepW = 1, kStepDQP = 2 };

template <class T, int NB>
bko_status launch_block_kernel(Step which, const Workspace &ws, int s, int init, hipStream_t st)
{
    const int64_t ldw = ws.ldw;
    const unsigned grid = grid_for(ldw);
    const bool f64 = sizeof(T) == 8;
    T *Dv = static_cast<T *>(ws.Dv), *Q = static_cast<T *>(ws.Q), *P = static_cast<T *>(ws.P);
    T *AP = static_cast<T *>(ws.AP), *W = static_cast<T *>(ws.W);
    const T *M1 = f64 ? reinterpret_cast<const T *>(ws.sm.M1) : reinterpret_cast<const T *>(ws.sm.M1f);
    const T *M2 = f64 ? reinterpret_cast<const T *>(ws.sm.M2) : reinterpret_cast<const T *>(ws.sm.M2f);
    const T *M3 = f64 ? reinterpret_cast<const T *>(ws.sm.M3) : reinterpret_cast<const T *>(ws.sm.M3f);
    const T *M4 = f64 ? reinterpret_cast<const T *>(ws.sm.M4) : reinterpret_cast<const T *>(ws.sm.M4f);
    const int sp = 16 * NB;
    const size_t mbytes = sizeof(T) * sp * (sp + 1);
    if (which == kStepGram) {
        TimedLaunch tl(kGram, st);
        hipLaunchKernelGGL((gram_kernel<T, NB>), dim3(grid), dim3(kThreads), 0, st, P, AP, ldw, s, ws.parts, ws.ctrl);
    } else if (which == kStepW) {
        TimedLaunch tl(kUpdate, st);
        hipLaunchKernelGGL((update_w_kernel<T, NB>), dim3(grid), dim3(kThreads), 0, st, Q, AP, W, M2, ldw, s, ws.parts,
                           ws.ctrl, init);
    } else {
        TimedLaunch tl(::bko::kUpdateDQP, st);
        hipLaunchKernelGGL((update_dqp_kernel<T, NB>), dim3(grid), dim3(kThreads), 3 * mbytes, st, Dv, P, Q, W, M1, M3,
                           M4, ldw, s, ws.ctrl);
    }
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class T>
bko_status launch_block(Step which, const Workspace &ws, int s, int init, hipStream_t st)
{
    switch (nb_for(s)) {
    case 1: return launch_block_kernel<T, 1>(which, ws, s, init, st);
    case 2: return launch_block_kernel<T, 2>(which, ws, s, init, st);
    case 3: return launch_block_kernel<T, 3>(which, ws, s, init, st);
    default: return launch_block_kernel<T, 4>(which, ws, s, init, st);
    }
}

// reduce the partials of the last Gram step, then factor (mode as factor_kernel)
bko_status launch_reduce_factor(const Workspace &ws, int s, double rel_thr, int mode, hipStream_t st)
{
    const int ss = s * s;
    const unsigned nparts = grid_for(ws.ldw);
    const unsigned rblocks = static_cast<unsigned>(std::min(kRedBlocks, ss));
    {
        TimedLaunch tl(kSmall, st);
        hipLaunchKernelGGL(gram_reduce_kernel, dim3(rblocks), dim3(kThreads), 0, st, ws.parts, static_cast<int>(nparts),
                           ss, ws.gram, ws.ctrl);
        BKO_HIP(hipGetLastError());
        // A, G, C (each padded by E <= 32), two pivot rows (padded) and columns
        const size_t lds = sizeof(double) * (4 * ss + 3 * 32 + 2 * (2 * s + 32) + 2 * s);
#define BKO_FACTOR(E, SP)                                                                                   \
    hipLaunchKernelGGL((factor_kernel<E, SP>), dim3(1), dim3(kFacThreads), lds, st, ws.gram, s, rel_thr, ws.sm, \
                       ws.ctrl, mode)
        const int e = factor_segment(s);
        if (s <= 8) BKO_FACTOR(1, 8);
        else if (s <= 16 && e == 1) BKO_FACTOR(1, 16);
        else if (s <= 16) BKO_FACTOR(2, 16);
        else if (s <= 32 && e == 4) BKO_FACTOR(4, 32);
        else if (s <= 32) BKO_FACTOR(8, 32);
        else if (e == 16) BKO_FACTOR(16, 0);
        else BKO_FACTOR(32, 0);
#undef BKO_FACTOR
        BKO_HIP(hipGetLastError());
    }
    return BKO_OK;
}

// Column norms of an FP64 n x s block, returned on the host.
bko_status host_colnorms(const double *A, int64_t lda, int64_t n, int s, double *colparts, std::vector<double> &out,
                         hipStream_t st)
{
    const int chunks = static_cast<int>(std::min<int64_t>(128, (n + 4095) / 4096));
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
// th: per-column absolute residual targets.
template <class T>
bko_status inner_solve(const Operator &op, int s, const Workspace &ws, const std::vector<double> &th, int budget,
                       int &iters_out, int &deflated_out, bool &all_deflated, hipStream_t st)
{
    const int64_t n = op.n, ldw = ws.ldw;
    const bool f64 = sizeof(T) == 8;
    const double rel_thr = f64 ? 1e-13 : 1e-12;
    const size_t blkv = sizeof(T) * static_cast<size_t>(ldw) * s;
    const size_t ss = static_cast<size_t>(s) * s;
    bko_status rc;

    // fresh state: blocks zero (padding rows stay zero), C = I, M1 = 0
    for (void *b : {ws.Dv, ws.Q, ws.P, ws.AP, ws.W})
        if ((rc = launch_zero(b, blkv, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(ws.ctrl, sizeof(int) * 64, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(ws.sm.M1, sizeof(double) * ss, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(ws.sm.M1f, sizeof(float) * ss, st)) != BKO_OK) return rc;
    hipLaunchKernelGGL(set_identity_kernel, dim3(1), dim3(256), 0, st, ws.sm.C, s);
    BKO_HIP(hipGetLastError());
    std::vector<double> thp(kMaxS, 0.0);
    std::copy(th.begin(), th.end(), thp.begin());
    BKO_HIP(hipMemcpyAsync(ws.sm.th, thp.data(), sizeof(double) * kMaxS, hipMemcpyHostToDevice, st));
    const unsigned rblocks = static_cast<unsigned>((n + 255) / 256);
    hipLaunchKernelGGL((cast_in_kernel<T>), dim3(rblocks), dim3(256), 0, st, ws.R64, ldw, static_cast<T *>(ws.W), ldw,
                       n, s);
    BKO_HIP(hipGetLastError());
    // first QR of the residual, then Q = W S^+, P = Q (P is zero), D = 0 (M1 = 0)
    if ((rc = launch_block<T>(kStepW, ws, s, 1, st)) != BKO_OK) return rc;
    if ((rc = launch_reduce_factor(ws, s, rel_thr, 2, st)) != BKO_OK) return rc;
    if ((rc = launch_block<T>(kStepDQP, ws, s, 0, st)) != BKO_OK) return rc;

    const bko_dtype vt = f64 ? BKO_F64 : BKO_F32;
    int h_ctrl[8] = {0};
    int launched = 0;
    int chunk = 4;
    while (true) {
        const int todo = std::min(chunk, budget - launched);
        for (int it = 0; it < todo; ++it) {
            {
                TimedLaunch tl(kSpmm, st);
                if ((rc = launch_stencil(op, s, ws.P, ldw, vt, ws.AP, ldw, vt, vt, nullptr, 0, st, ws.ctrl + kConverged,
                                         ws.ctrl + kStop)) != BKO_OK)
                    return rc;
            }
            if ((rc = launch_block<T>(kStepGram, ws, s, 0, st)) != BKO_OK) return rc;
            if ((rc = launch_reduce_factor(ws, s, rel_thr, 0, st)) != BKO_OK) return rc;
            if ((rc = launch_block<T>(kStepW, ws, s, 0, st)) != BKO_OK) return rc;
            if ((rc = launch_reduce_factor(ws, s, rel_thr, 1, st)) != BKO_OK) return rc;
            if ((rc = launch_block<T>(kStepDQP, ws, s, 0, st)) != BKO_OK) return rc;
        }
        launched += todo;
        BKO_HIP(hipMemcpyAsync(h_ctrl, ws.ctrl, sizeof(h_ctrl), hipMemcpyDeviceToHost, st));
        BKO_HIP(hipStreamSynchronize(st));
        if (h_ctrl[kConverged] || launched >= budget) break;
        chunk = std::min(chunk * 2, 64);
    }
    iters_out = h_ctrl[kIters];
    deflated_out = h_ctrl[kDeflated];
    all_deflated = h_ctrl[kAllDeflated] != 0;
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
    // LDS needed by the FP64 update kernel at this s
    {
        const size_t sp = 16 * static_cast<size_t>(nb_for(s));
        const size_t need = 3 * (compute == BKO_F64 ? 8 : 4) * sp * (sp + 1);
        const size_t cap = device_max_lds();
        if (need > cap || sizeof(double) * 4 * s * s > cap) {
            set_error("s = %d needs %zu bytes of LDS per workgroup in this precision; the device grants %zu", s, need,
                      cap);
            return BKO_EINVAL;
        }
    }
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
        // R = B - A X in FP64 (the cast into the inner blocks reads rows < n)
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
