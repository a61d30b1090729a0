// Block Krylov solve of A X = B for s right-hand sides sharing one heat
// operator (Sec. III-A, Eq. (4)), for one chip or for a batch of chips of
// different grids at once (the chip index j of Eq. (4) runs over the batch).
//
// The paper names block CG without fixing a variant.  This is the retooled
// block CG that carries an orthonormal residual basis Q (R = Q C) so that
// columns converging at different rates do not make the s x s systems ill
// conditioned, with rank-revealing factorisations that drop linearly
// dependent directions instead of breaking down.  One iteration, with P the
// search block:
//     AP    = A P                                  (stencil product)
//     delta = P^T AP                               (FP64 Gram)
//     W'    = Q - AP delta^+                       (next residual basis)
//     W'^T W' = S^T S  (S upper triangular)        (Cholesky QR, FP64)
//     D    += P delta^+ C ;  Q' = W' S^+ ;  P = Q' + P S^T ;  C = S C
// and ||r_j|| = ||C e_j||, so convergence is read off C without a pass over
// the residual.  Q is never stored: the kernels form Q = W S^+ from the W of
// the previous step when they need it (W is updated in place).
//
// Grouped launches: every kernel of an iteration covers all chips of the
// batch in one launch.  A table maps each workgroup to its chip, and each
// chip's parameters (grid, coefficient and block pointers, small matrices,
// control words) sit in a device array that the kernels read; a chip that
// has converged makes its workgroups return at once.  Kernels per iteration,
// all on one stream with no host round trip (the kernel boundary is the only
// grid-wide synchronisation: an in-kernel fence per workgroup costs far more
// on this chip than the boundary):
//   spmm_gram   AP = A P (matrix-free stencil), with P and AP staged in LDS
//               and their per-workgroup P^T AP partials on the FP64 matrix
//               cores
//   reduce      the partials summed entry by entry, in index order
//   factor      one workgroup per chip: delta^+ and delta^+ C
//   update_w    W <- W S^+ - AP delta^+ on the matrix cores, and the W^T W
//               partials from the same registers
//   reduce
//   factor      W^T W = S^T S, C <- S C, convergence test
//   update_dqp  D += P delta^+ C, P = W S^+ + P S^T
// The iteration chunks between convergence checks can be replayed from
// captured HIP graphs.
//
// The s x s factorisations are an LDL^T elimination of [G | I] without
// pivoting in which a pivot below a relative threshold deactivates its index
// (its row and column of every derived matrix are zero).
//
// Storage: the N x s blocks are FP64 or FP32 (compute = BKO_F32); Gram
// matrices, factorisations, small matrices and the outer residual are FP64.
// An outer loop forms R = B - A X in FP64, runs the block iteration on
// A D = R, adds D to X, and stops when max_j ||r_j|| / ||b_j|| <= tol (FP64
// iterative refinement in the mixed-precision mode).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;      // row kernels
constexpr int kFacThreads = 256;   // factorisation kernel
constexpr int kMaxS = 64;
constexpr int kRedBlocks = 128;    // reducer workgroups per chip
constexpr int kTileRows = 256;     // rows per tile of the row kernels (4 waves x 64)
constexpr int kCtrlInts = 16;      // control words per chip

// ------------------------------------------------------------------ layout

enum Ctrl { kConverged = 0, kStop = 1, kIters = 2, kDeflated = 3, kAllDeflated = 4, kActive = 5 };

struct Small {
    // FP64, row-major s x s: M[k][j] maps input column k to output column j
    double *C, *M1, *M2, *M3, *M4, *th;
    // FP32 copies for the FP32 block kernels
    float *M1f, *M2f, *M3f, *M4f;
};

// Device view of Small with global-memory pointers.
struct SmallG;

// What a grouped kernel knows about one chip.
struct ChipDev {
    // operator: coefficients in the block precision, and in FP64
    const void *cdiag, *cwx, *cwy, *cwz;   // the iterated operator (S A S under Jacobi)
    const double *d64, *x64, *y64, *z64;  // A, for the FP64 residual
    const double *scale;                  // S = diag(A)^(-1/2) under Jacobi, else null
    int nx, ny, nz, wgs;   // wgs: workgroups of the row kernels for this chip
    int64_t n, ldw;        // cells, padded rows of every internal block
    int wg_base, pad;
    // caller arrays (FP64, column major)
    const double *B;
    int64_t ldb;
    double *X;
    int64_t ldx;
    const double *X0;
    int64_t ldx0;
    // inner blocks (block precision) and the FP64 residual
    void *Dv, *P, *AP, *W;
    double *R64;
    Small sm;
    double *parts;  // [wgs][s][s] Gram partials, also [wgs][s] or [wgs][2 s] column sums
    double *gram;   // [s][s]
    double *norms;  // [kMaxS] squared column norms
    int *ctrl;      // kCtrlInts control words
};

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

// Pointers read from the chip records are generic to the compiler; marking
// them as global memory lets it emit global (not flat) loads and stores.
template <class T> using gptr = T __attribute__((address_space(1))) *;
template <class T> __device__ __forceinline__ gptr<T> glb(T *p) { return (gptr<T>)p; }

struct SmallG {
    gptr<double> C, M1, M2, M3, M4, th;
    gptr<float> M1f, M2f, M3f, M4f;
    __device__ explicit SmallG(const Small &m)
        : C(glb(m.C)), M1(glb(m.M1)), M2(glb(m.M2)), M3(glb(m.M3)), M4(glb(m.M4)), th(glb(m.th)), M1f(glb(m.M1f)),
          M2f(glb(m.M2f)), M3f(glb(m.M3f)), M4f(glb(m.M4f))
    {
    }
};

// Chip of this workgroup and the workgroup's index within the chip.  A
// layout of one chip passes no table (one dependent load fewer at the start
// of every row kernel).
__device__ inline int chip_index(const uint16_t *tab) { return tab ? tab[blockIdx.x] : 0; }
__device__ inline const ChipDev &chip_of(const ChipDev *cds, const uint16_t *tab, int &local)
{
    if (!tab) {
        local = static_cast<int>(blockIdx.x);
        return cds[0];
    }
    const ChipDev &cd = cds[tab[blockIdx.x]];
    local = static_cast<int>(blockIdx.x) - cd.wg_base;
    return cd;
}

// The tiles (of `unit` consecutive cells: 256, or one LDS stage) a
// workgroup of the stencil + Gram product takes, in order.  When the chip's
// planes are whole tiles, the tiles are numbered
// z-major (in-plane tile q, plane l -> q nz + l) and each workgroup takes a
// run of consecutive numbers in the XCD-contiguous workgroup order, so it
// walks consecutive planes of one in-plane tile: the neighbours one plane
// away are the tiles it has just read or reads next, and the workgroups
// beside it on the same XCD hold the neighbouring rows, all served from that
// XCD's L2.  Otherwise the tiles are dealt round-robin.
struct TileWalk {
    int64_t i0, i1, step, tp;
    int nz;
    bool zmajor;
    __device__ TileWalk(int local, int wgs, int64_t ntiles, int64_t plane, int nz_, int unit = kTileRows)
    {
        nz = nz_;
        tp = plane / unit;
        zmajor = plane % unit == 0 && tp * nz == ntiles;
        if (zmajor) {
            const int64_t per = (ntiles + wgs - 1) / wgs;
            i0 = static_cast<int64_t>(remap_block(static_cast<uint32_t>(local), static_cast<uint32_t>(wgs))) * per;
            i1 = i0 + per < ntiles ? i0 + per : ntiles;
            step = 1;
        } else {
            i0 = local;
            i1 = ntiles;
            step = wgs;
        }
    }
    __device__ int64_t tile(int64_t i) const { return zmajor ? i / nz + tp * (i % nz) : i; }
};

// ------------------------------------------------------------------ Gram partials

// Row and column block of Gram block q: the upper blocks (a <= b) in order
// when kSym, else all blocks row by row.
template <int NB, bool kSym> __device__ __forceinline__ void gram_block(int q, int &a, int &b)
{
    if (!kSym) {
        a = q / NB;
        b = q % NB;
        return;
    }
    a = 0;
    while (q >= NB - a) {
        q -= NB - a;
        ++a;
    }
    b = a + q;
}

// LDS doubles publish_partial needs: each wave stores CB blocks per round.
template <int kNT> __host__ __device__ constexpr int publish_lds(int cb) { return cb * (kNT / 64) * 4 * 64; }

// Sum the waves' 16x16 FP64 Gram blocks and write the s x s partial to out.
// Each round, every wave stores CB of its blocks to its own LDS slots (lane
// fastest, no bank conflicts); after one barrier wave c % NW sums block c
// over the waves in wave order and writes it.  kSym: only upper blocks were
// formed; each is also written transposed.  lds: publish_lds<kNT>(CB)
// doubles.
template <int NB, bool kSym, int NBLK, int kNT = kThreads, int CB = (NBLK < 4 ? NBLK : 4)>
__device__ void publish_partial(const d4 (&g)[NBLK], int s, double *lds, gptr<double> out)
{
    constexpr int NW = kNT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int q0 = 0; q0 < NBLK; q0 += CB) {
        if (q0 > 0) __syncthreads();
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (q0 + c < NBLK) {
#pragma unroll
                for (int r = 0; r < 4; ++r) lds[((wave * CB + c) * 4 + r) * 64 + lane] = g[q0 + c][r];
            }
        __syncthreads();
        for (int c = wave; c < CB && q0 + c < NBLK; c += NW) {
            int a, b;
            gram_block<NB, kSym>(q0 + c, a, b);
            const int j = b * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = lds[(c * 4 + r) * 64 + lane];
#pragma unroll
                for (int wv = 1; wv < NW; ++wv) v += lds[((wv * CB + c) * 4 + r) * 64 + lane];
                const int i = a * 16 + mfma_row<true>(lg, r);
                if (i < s && j < s) {
                    out[i * s + j] = v;
                    if (kSym && a != b) out[j * s + i] = v;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ stencil product + Gram

// Consecutive cells one 16-byte access covers.
template <class T> __host__ __device__ constexpr int vec_cells() { return 16 / static_cast<int>(sizeof(T)); }

// Rows of a 256-row tile staged in LDS at once: the whole tile when P and AP
// of all 16 NB columns fit in 70 KB (two workgroups per CU), else half.
// Staged columns are padded by one 16-byte vector.
template <class T, int NB> __host__ __device__ constexpr int stage_rows()
{
    return 2 * 16 * NB * (kTileRows + vec_cells<T>()) * static_cast<int>(sizeof(T)) <= 70 * 1024 ? kTileRows
                                                                                                 : kTileRows / 2;
}

template <class T, int NB> __host__ __device__ constexpr int stage_ld() { return stage_rows<T, NB>() + vec_cells<T>(); }

template <class T, int NB> __host__ __device__ constexpr size_t spmm_gram_lds()
{
    return 2 * sizeof(T) * 16 * NB * stage_ld<T, NB>();
}

// AP = A P for the chip's tiles, and the chip's P^T AP partial of this
// workgroup.  Stencil phase: thread (cell, column class) forms the 7-point
// product of its cell for every column of its class, writes AP, and stages
// P and AP in LDS; Gram phase: each wave takes a quarter of the staged rows
// on the FP64 matrix cores, forming only the upper 16 x 16 blocks (P^T A P
// is symmetric; the partial is written with its transpose).
constexpr int kSpThreads = 256;  // stencil + Gram kernel (eight-wave workgroups measured slower)
// For s > 32 the stencil + Gram kernels are held to two waves per SIMD: left
// to itself the compiler spends registers on one (measured 25 % slower).

template <class T, int NB>
__global__ __launch_bounds__(kSpThreads, (NB > 2 ? 2 : 1)) void spmm_gram_kernel(const ChipDev *__restrict__ cds,
                                                                                  const uint16_t *__restrict__ tab,
                                                                                  int s)
{
    constexpr int TR = stage_rows<T, NB>();
    constexpr int SP = 16 * NB;
    constexpr int LD = stage_ld<T, NB>();
    constexpr int CSTEP = kSpThreads / TR;  // column classes
    constexpr int NW = kSpThreads / 64;     // waves
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    gptr<int> ctrl = glb(cd.ctrl);
    if (ctrl[kConverged]) {
        // the iteration before this one converged: tell the later kernels
        if (local == 0 && threadIdx.x == 0) ctrl[kStop] = 1;
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    T *Ps = reinterpret_cast<T *>(smem);
    T *APs = Ps + SP * LD;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    // columns s .. SP of the staged tiles stay zero
    for (int e = s * LD + tid; e < SP * LD; e += kSpThreads) {
        Ps[e] = T(0);
        APs[e] = T(0);
    }
    const gptr<const T> __restrict__ P = glb(static_cast<const T *>(cd.P));
    const gptr<T> __restrict__ AP = glb(static_cast<T *>(cd.AP));
    const gptr<const T> __restrict__ cdiag = glb(static_cast<const T *>(cd.cdiag));
    const gptr<const T> __restrict__ cwx = glb(static_cast<const T *>(cd.cwx));
    const gptr<const T> __restrict__ cwy = glb(static_cast<const T *>(cd.cwy));
    const gptr<const T> __restrict__ cwz = glb(static_cast<const T *>(cd.cwz));
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int64_t n = cd.n, ldw = cd.ldw;
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int cell = tid % TR, cls = tid / TR;

    d4 acc[NB * (NB + 1) / 2];  // upper blocks of P^T AP (symmetric)
#pragma unroll
    for (int q = 0; q < NB * (NB + 1) / 2; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t ntiles = ldw / kTileRows;
    const TileWalk walk(local, wgs, ntiles, plane, nz);
    for (int64_t it = walk.i0; it < walk.i1; it += walk.step) {
        const int64_t tile = walk.tile(it);
        for (int half = 0; half < kTileRows / TR; ++half) {
            const int64_t a = tile * kTileRows + half * TR + cell;
            if (a < n) {
                const int i = static_cast<int>(a % nx);
                const int64_t q = a / nx;
                const int j = static_cast<int>(q % ny);
                const int l = static_cast<int>(q / ny);
                // a missing neighbour reads the cell itself with a zero coupling
                const int64_t oxm = i > 0 ? -1 : 0, oxp = i < nx - 1 ? 1 : 0;
                const int64_t oym = j > 0 ? -static_cast<int64_t>(nx) : 0, oyp = j < ny - 1 ? nx : 0;
                const int64_t ozm = l > 0 ? -plane : 0, ozp = l < nz - 1 ? plane : 0;
                const T d = cdiag[a];
                const T cxp = cwx[a], cxm = i > 0 ? cwx[a - 1] : T(0);
                const T cyp = cwy[a], cym = j > 0 ? cwy[a - nx] : T(0);
                const T czp = cwz[a], czm = l > 0 ? cwz[a - plane] : T(0);
#pragma unroll 4
                for (int c = cls; c < s; c += CSTEP) {
                    const gptr<const T> x = P + c * ldw + a;
                    const T xc = x[0];
                    const T nb = cxm * x[oxm] + cxp * x[oxp] + cym * x[oym] + cyp * x[oyp] + czm * x[ozm] + czp * x[ozp];
                    const T y = d * xc - nb;
                    AP[c * ldw + a] = y;
                    Ps[c * LD + cell] = xc;
                    APs[c * LD + cell] = y;
                }
            } else {
                // padding rows of the tile: zero in the Gram (AP keeps its zero padding)
                for (int c = cls; c < s; c += CSTEP) {
                    Ps[c * LD + cell] = T(0);
                    APs[c * LD + cell] = T(0);
                }
            }
            __syncthreads();
            // Gram phase: rows r + t feed MFMA step t for lane group lg (any
            // bijection of rows onto k slots works, since the product sums
            // over rows); each wave takes TR / NW rows
#pragma unroll
            for (int rb = 0; rb < TR / (16 * NW); ++rb) {
                const int r = wave * (TR / NW) + rb * 16 + lg * 4;
                double u[NB][4], v[NB][4];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int col = b * 16 + li;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        u[b][t] = static_cast<double>(Ps[col * LD + r + t]);
                        v[b][t] = static_cast<double>(APs[col * LD + r + t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int x = 0; x < NB; ++x)
#pragma unroll
                        for (int y = x; y < NB; ++y)
                            acc[ublock<NB>(x, y)] = mma64(u[x][t], v[y][t], acc[ublock<NB>(x, y)]);
            }
            __syncthreads();
        }
    }
    static_assert(spmm_gram_lds<T, NB>() >= sizeof(double) * publish_lds<kSpThreads>(NB * NB < 4 ? NB * NB : 4),
                  "publish_partial needs more LDS than the staged tiles");
    publish_partial<NB, true, NB * (NB + 1) / 2, kSpThreads>(acc, s, reinterpret_cast<double *>(smem),
                                                    glb(cd.parts) + static_cast<size_t>(local) * s * s);
}

// 16-byte vector of block elements.
template <class T> struct Vec16;
template <> struct Vec16<float> {
    using type = f4;
};
template <> struct Vec16<double> {
    typedef double d2 __attribute__((ext_vector_type(2)));
    using type = d2;
};

template <class T> __device__ __forceinline__ typename Vec16<T>::type ld16(gptr<const T> p)
{
    return *reinterpret_cast<gptr<const typename Vec16<T>::type>>(p);
}

// spmm_gram_kernel with V = 16 / sizeof(T) consecutive cells per thread, so
// that every access to P, AP, the coefficients and the LDS stage is one
// 16-byte operation (chips whose nx is a multiple of V: a group of V cells
// then lies in one x-row).  The x neighbours inside the group come from its
// own vector, the two outside it from scalar loads.  The unit of work is one
// LDS stage of TR rows, walked as TileWalk orders it; in a z-major walk of
// FP32 blocks with s > 32 (streamed from HBM) each thread keeps its vectors
// of the current plane and the plane above from one stage to the next
// (kCarry), so a run of planes reads each vector of P once for its own plane
// and as the z neighbours of the planes beside it.  For s > 32 the Gram
// blocks are shared out over the waves (kOwn): each wave accumulates whole
// upper 16 x 16 blocks over all staged rows, and the NBLK % 4 remaining
// blocks over a quarter of the rows each (summed through LDS at the end), so
// a wave holds at most four accumulator blocks; for s <= 32 each wave takes
// every block over a quarter of the rows.
template <class T, int NB>
__global__ __launch_bounds__(kSpThreads, (NB > 2 ? 2 : 1)) void spmm_gram_vec_kernel(const ChipDev *__restrict__ cds,
                                                                                      const uint16_t *__restrict__ tab,
                                                                                      int s)
{
    using VT = typename Vec16<T>::type;
    constexpr int V = vec_cells<T>();
    constexpr int TR = stage_rows<T, NB>();
    constexpr int SP = 16 * NB;
    constexpr int LD = stage_ld<T, NB>();
    constexpr int TPC = TR / V;              // threads per column class
    constexpr int CSTEP = kSpThreads / TPC;  // column classes
    constexpr int NCOL = (SP + CSTEP - 1) / CSTEP;  // columns per thread at most
    constexpr int NW = kSpThreads / 64;
    constexpr int NBLK = NB * (NB + 1) / 2;
    constexpr int FB = NBLK / NW;  // whole Gram blocks per wave
    constexpr int RB = NBLK % NW;  // blocks shared by every wave (a quarter of the rows each)
    constexpr bool kCarry = sizeof(T) == 4 && NB > 2;
    constexpr bool kOwn = NB > 2;  // Gram blocks owned by waves
    static_assert(kSpThreads % TPC == 0 && (LD * sizeof(T)) % 16 == 0, "vector staging");
    static_assert(TR % (16 * NW) == 0, "row quarters of the Gram");
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    gptr<int> ctrl = glb(cd.ctrl);
    if (ctrl[kConverged]) {
        if (local == 0 && threadIdx.x == 0) ctrl[kStop] = 1;
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    T *Ps = reinterpret_cast<T *>(smem);
    T *APs = Ps + SP * LD;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    for (int e = s * LD + tid; e < SP * LD; e += kSpThreads) {
        Ps[e] = T(0);
        APs[e] = T(0);
    }
    const gptr<const T> __restrict__ P = glb(static_cast<const T *>(cd.P));
    const gptr<T> __restrict__ AP = glb(static_cast<T *>(cd.AP));
    const gptr<const T> __restrict__ cdiag = glb(static_cast<const T *>(cd.cdiag));
    const gptr<const T> __restrict__ cwx = glb(static_cast<const T *>(cd.cwx));
    const gptr<const T> __restrict__ cwy = glb(static_cast<const T *>(cd.cwy));
    const gptr<const T> __restrict__ cwz = glb(static_cast<const T *>(cd.cwz));
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int64_t n = cd.n, ldw = cd.ldw;
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int cell = (tid % TPC) * V, cls = tid / TPC;
    const VT zero = VT(T(0));

    // s > 32: this wave's Gram blocks are whole blocks wave + NW f and a
    // quarter of the rows of each shared block NW FB + r; s <= 32: every
    // block over a quarter of the rows
    constexpr int NACC = kOwn ? FB + RB : NBLK;
    int ga[NACC], gb[NACC];
    if constexpr (kOwn) {
#pragma unroll
        for (int f = 0; f < FB; ++f) gram_block<NB, true>(wave + NW * f, ga[f], gb[f]);
#pragma unroll
        for (int r = 0; r < RB; ++r) gram_block<NB, true>(NW * FB + r, ga[FB + r], gb[FB + r]);
    }
    d4 acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

    VT c0[kCarry ? NCOL : 1], c1[kCarry ? NCOL : 1];  // plane below and this plane, carried
    const TileWalk walk(local, wgs, ldw / TR, plane, nz, TR);
    for (int64_t it = walk.i0; it < walk.i1; it += walk.step) {
        const int64_t a = walk.tile(it) * TR + cell;
        // the previous stage of this workgroup was the same rows one plane down
        const bool cont = kCarry && walk.zmajor && it != walk.i0 && it % nz != 0;
        if (a < n) {
            const int i0 = static_cast<int>(a % nx);
            const int64_t q = a / nx;
            const int j = static_cast<int>(q % ny);
            const int l = static_cast<int>(q / ny);
            // a missing neighbour reads the group itself with a zero coupling
            const int64_t oxl = i0 > 0 ? -1 : 0, oxr = i0 + V < nx ? V : V - 1;
            const int64_t oym = j > 0 ? -static_cast<int64_t>(nx) : 0, oyp = j < ny - 1 ? nx : 0;
            const int64_t ozm = l > 0 ? -plane : 0, ozp = l < nz - 1 ? plane : 0;
            const VT d = ld16(cdiag + a), cxp = ld16(cwx + a), cyp = ld16(cwy + a), czp = ld16(cwz + a);
            const VT cym = j > 0 ? ld16(cwy + a - nx) : zero;
            const VT czm = l > 0 ? ld16(cwz + a - plane) : zero;
            VT cxm;
            cxm[0] = i0 > 0 ? cwx[a - 1] : T(0);
#pragma unroll
            for (int e = 1; e < V; ++e) cxm[e] = cxp[e - 1];
            auto column = [&](int c, VT &k0, VT &k1) __attribute__((always_inline)) {
                const gptr<const T> x = P + c * ldw + a;
                VT xc, xzm;
                if (cont) {
                    xzm = k0;
                    xc = k1;
                } else {
                    xc = ld16(x);
                    xzm = ld16(x + ozm);
                }
                const VT xym = ld16(x + oym), xyp = ld16(x + oyp), xzp = ld16(x + ozp);
                const T xl = x[oxl], xr = x[oxr];
                VT y;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const T left = e == 0 ? xl : xc[e > 0 ? e - 1 : 0];
                    const T right = e == V - 1 ? xr : xc[e < V - 1 ? e + 1 : 0];
                    const T nb = cxm[e] * left + cxp[e] * right + cym[e] * xym[e] + cyp[e] * xyp[e] +
                                 czm[e] * xzm[e] + czp[e] * xzp[e];
                    y[e] = d[e] * xc[e] - nb;
                }
                *reinterpret_cast<gptr<VT>>(AP + c * ldw + a) = y;
                *reinterpret_cast<VT *>(Ps + c * LD + cell) = xc;
                *reinterpret_cast<VT *>(APs + c * LD + cell) = y;
                k0 = xc;
                k1 = xzp;
            };
            if constexpr (kCarry) {
#pragma unroll
                for (int k = 0; k < NCOL; ++k)
                    if (cls + k * CSTEP < s) column(cls + k * CSTEP, c0[k], c1[k]);
            } else {
#pragma unroll 2
                for (int c = cls; c < s; c += CSTEP) column(c, c0[0], c1[0]);
            }
        } else {
            // padding rows of the stage: zero in the Gram (AP keeps its zero padding)
            for (int c = cls; c < s; c += CSTEP) {
                *reinterpret_cast<VT *>(Ps + c * LD + cell) = zero;
                *reinterpret_cast<VT *>(APs + c * LD + cell) = zero;
            }
        }
        __syncthreads();
        if constexpr (kOwn) {
            // P^T AP over the staged rows: row k0 + lg is the k slot of lane group lg
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const T *pa = Ps + (ga[f] * 16 + li) * LD + lg, *pb = APs + (gb[f] * 16 + li) * LD + lg;
#pragma unroll 8
                for (int k0 = 0; k0 < TR; k0 += 4)
                    acc[f] = mma64(static_cast<double>(pa[k0]), static_cast<double>(pb[k0]), acc[f]);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int rows0 = wave * (TR / NW);
                const T *pa = Ps + (ga[FB + r] * 16 + li) * LD + rows0 + lg;
                const T *pb = APs + (gb[FB + r] * 16 + li) * LD + rows0 + lg;
#pragma unroll 8
                for (int k0 = 0; k0 < TR / NW; k0 += 4)
                    acc[FB + r] = mma64(static_cast<double>(pa[k0]), static_cast<double>(pb[k0]), acc[FB + r]);
            }
        } else {
            // every block over this wave's quarter of the staged rows: rows
            // r + t feed matrix-core step t for lane group lg
#pragma unroll
            for (int rb = 0; rb < TR / (16 * NW); ++rb) {
                const int r = wave * (TR / NW) + rb * 16 + lg * 4;
                double u[NB][4], v[NB][4];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int col = b * 16 + li;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        u[b][t] = static_cast<double>(Ps[col * LD + r + t]);
                        v[b][t] = static_cast<double>(APs[col * LD + r + t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int x = 0; x < NB; ++x)
#pragma unroll
                        for (int y = x; y < NB; ++y)
                            acc[ublock<NB>(x, y)] = mma64(u[x][t], v[y][t], acc[ublock<NB>(x, y)]);
            }
        }
        __syncthreads();
    }
    if constexpr (!kOwn) {
        static_assert(spmm_gram_lds<T, NB>() >= sizeof(double) * publish_lds<kSpThreads>(NB * NB < 4 ? NB * NB : 4),
                      "publish_partial needs more LDS than the staged tiles");
        publish_partial<NB, true, NBLK, kSpThreads>(acc, s, reinterpret_cast<double *>(smem),
                                                    glb(cd.parts) + static_cast<size_t>(local) * s * s);
        return;
    } else {
        // publish: whole blocks by their wave; the shared blocks summed through LDS
        const gptr<double> out = glb(cd.parts) + static_cast<size_t>(local) * s * s;
        auto put = [&](int ab, int bb, const d4 &v) {
            const int jj = bb * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ii = ab * 16 + mfma_row<true>(lg, r);
                if (ii < s && jj < s) {
                    out[ii * s + jj] = v[r];
                    if (ab != bb) out[jj * s + ii] = v[r];
                }
            }
        };
#pragma unroll
        for (int f = 0; f < FB; ++f) put(ga[f], gb[f], acc[f]);
        if constexpr (RB > 0) {
            static_assert(spmm_gram_lds<T, NB>() >= sizeof(double) * RB * NW * 4 * 64, "LDS for the shared blocks");
            double *xs = reinterpret_cast<double *>(smem);
            __syncthreads();  // the stage is dead (also when this workgroup had no rows)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) xs[((r * NW + wave) * 4 + e) * 64 + lane] = acc[FB + r][e];
            __syncthreads();
            for (int r = wave; r < RB; r += NW) {
                d4 v = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int w = 0; w < NW; ++w)
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] += xs[((r * NW + w) * 4 + e) * 64 + lane];
                put(ga[FB + r], gb[FB + r], v);
            }
        }
    }
}

// gram = sum over the chip's partials, entry by entry in index order
// (grid: kRedBlocks x chips).
__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(const ChipDev *__restrict__ cds, int ss)
{
    const ChipDev &cd = cds[blockIdx.y];
    const gptr<const double> __restrict__ parts = glb(static_cast<const double *>(cd.parts));
    const int nparts = cd.wgs;
    const gptr<const int> ctrl = glb(cd.ctrl);
    __shared__ double sh[kThreads];
    const int per = (ss + gridDim.x - 1) / gridDim.x;  // entries of this workgroup (<= 64)
    const int slices = kThreads / per;
    const int tid = threadIdx.x;
    const int le = tid % per, sl = tid / per;
    const int e = blockIdx.x * per + le;
    double a = 0.0;
    // the control word is tested after the partials are summed, so that its
    // latency overlaps their loads (a converged chip's reduction reads them
    // for nothing and writes nothing); read with a vector load (the empty asm
    // hides that the offset is uniform), so that waiting for the chip's
    // pointers does not wait for it too
    int zo = 0;
    asm volatile("" : "+v"(zo));
    const int stop = ctrl[kConverged + zo];
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
    if (stop) return;
    sh[tid] = a;
    __syncthreads();
    if (sl == 0 && e < ss) {
        double tot = 0.0;
        for (int q = 0; q < slices; ++q) tot += sh[q * per + le];
        glb(cd.gram)[e] = tot;
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

// 1 / p from the hardware reciprocal estimate and two Newton steps (each
// squares the relative error), for the pivots on the elimination's serial
// path; within an ulp or two of the correctly rounded quotient for the
// normal, positive pivots it is used on.
__device__ __forceinline__ double recip(double p)
{
    double r = __builtin_amdgcn_rcp(p);
    r = fma(r, fma(-p, r, 1.0), r);
    return fma(r, fma(-p, r, 1.0), r);
}

// Masked LDL^T elimination of [G | I] by one wavefront, for s <= SP <= 32:
// lane c holds column c of the 2 SP columns in registers; each pivot row of
// the column is broadcast with readlane, so no LDS traffic or barrier per
// pivot.  Indices s <= i < SP are decoupled padding with pivot gmax.  g is
// an LDS copy of the Gram with row stride ld; the result (A[i][j], j < 2s:
// left half U, right half E) goes to LDS and may overwrite g (every read of
// g precedes the first write).  gmax_ext >= 0 replaces the block's own largest
// diagonal in the deactivation threshold; ldA > 0 and roff place the output
// rows (stride ldA) and the right half (from column roff) in a larger array.
// kSym: g is exactly symmetric already, so its transposed reads (bank
// conflicts at a row stride of 64 doubles) are skipped; the result is the
// same bit for bit, since (x + x) / 2 = x.
template <int SP, bool kSym = false>
__device__ __forceinline__ void wave_eliminate(const double *g, int ld, int s, double rel_thr, double *A, int *active,
                                               double gmax_ext = -1.0, int ldA = 0, int roff = 0)
{
    const int lane = threadIdx.x & 63;
    const int w = ldA > 0 ? ldA : 2 * s;  // output row stride
    const int ro = ldA > 0 ? roff : s;    // output column of the right half's first column
    // every lane reads (at a clamped index) so that the reads issue back to
    // back, with no branch between them
    const int lc = lane < s ? lane : 0;
    double x[SP], y[SP];
#pragma unroll
    for (int i = 0; i < SP; ++i) {
        const int ic = i < s ? i : 0;
        x[i] = g[ic * ld + lc];
        if constexpr (!kSym) y[i] = g[lc * ld + ic];
    }
    double gmax = g[lc * ld + lc];
    gmax = lane < s ? gmax : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off));
    if (gmax_ext >= 0.0) gmax = gmax_ext;
    const double thr = rel_thr * gmax;
    double a[SP];
#pragma unroll
    for (int i = 0; i < SP; ++i) {
        const double gi = kSym ? x[i] : 0.5 * (x[i] + y[i]);
        const double left = (i < s && lane < s) ? gi : (i == lane ? gmax : 0.0);
        const double right = (i == lane - SP) ? 1.0 : 0.0;
        a[i] = lane < SP ? left : right;
    }
#pragma unroll
    for (int k = 0; k < SP; ++k) {
        const double p = readlane_f64(a[k], k);
        const bool act = p > thr && isfinite(p);
        // this column's pivot-row entry, scaled; zero when the pivot is inactive
        const double m = act ? -a[k] * recip(p) : 0.0;
#pragma unroll
        for (int i = k + 1; i < SP; ++i) a[i] = fma(readlane_f64(a[i], k), m, a[i]);
        if (lane == 0 && k < s) active[k] = act ? 1 : 0;
    }
    const int col = lane < SP ? (lane < s ? lane : -1) : (lane - SP < s ? ro + lane - SP : -1);
    if (lane < 2 * SP && col >= 0) {
#pragma unroll
        for (int i = 0; i < SP; ++i)
            if (i < s) A[i * w + col] = a[i];
    }
}

// out(i, j, sum_k fa(i, k) fb(k, j)) for an s x s product (s <= 4 KT) on the
// FP64 matrix cores, by a workgroup that factors a Gram (the factorisation
// kernel, or every workgroup of a fused update).  The wave index is made
// scalar, so block indices and k ranges are uniform; each wave gathers the
// operands of all KT k steps of two output blocks (reads at clamped indices,
// out-of-range and skipped terms selected to zero afterwards, so that the
// reads issue back to back with no branch between them) before the first
// matrix-core step, then runs the two accumulation chains interleaved and
// unconditionally (a conditional step makes the compiler copy the
// accumulator around it).  fa and fb must read valid memory for every index
// below s.  kfirst(bi, bj) is the first k step (of 4) that can be nonzero
// for output block (bi, bj), for triangular operands; the terms before it
// are zero either way.
template <int KT, class FA, class FB, class FO, class FK>
__device__ __forceinline__ void small_gemm(int s, FA fa, FB fb, FO out, FK kfirst)
{
    constexpr int NW = kFacThreads / 64;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int li = lane & 15, lg = lane >> 4;
    const int nb = (s + 15) / 16, nbb = nb * nb;
    for (int blk = wave; blk < nbb; blk += 2 * NW) {
        const bool two = blk + NW < nbb;
        int bi[2], bj[2];
        double av[2][KT], bv[2][KT];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int b = h == 0 || two ? blk + h * NW : blk;
            bi[h] = b / nb;
            bj[h] = b % nb;
            const int k0 = kfirst(bi[h], bj[h]);
            const int i = bi[h] * 16 + li, j = bj[h] * 16 + li;
            const int ic = i < s ? i : s - 1, jc = j < s ? j : s - 1;
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int k = 4 * t + lg;
                const int kc = k < s ? k : s - 1;
                const double va = fa(ic, kc), vb = fb(kc, jc);
                const bool kin = k < s && t >= k0;
                av[h][t] = (i < s && kin) ? va : 0.0;
                bv[h][t] = (j < s && kin) ? vb : 0.0;
            }
        }
        d4 acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
        if (two) {
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                acc[0] = mma64(av[0][t], bv[0][t], acc[0]);
                acc[1] = mma64(av[1][t], bv[1][t], acc[1]);
            }
        } else {
#pragma unroll
            for (int t = 0; t < KT; ++t) acc[0] = mma64(av[0][t], bv[0][t], acc[0]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !two) continue;
            const int j = bj[h] * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int io = bi[h] * 16 + mfma_row<true>(lg, r);
                if (io < s && j < s) out(io, j, acc[h][r]);
            }
        }
    }
}
template <int KT, class FA, class FB, class FO>
__device__ __forceinline__ void small_gemm(int s, FA fa, FB fb, FO out)
{
    small_gemm<KT>(s, fa, fb, out, [](int, int) { return 0; });
}

// LDS of a workgroup that factors its chip's s x s Gram itself (s <= 32).
struct FacScratch {
    double A[2 * 32 * 32];  // the Gram (row stride s + 1), then [U | E] after the elimination, s x 2s
    double G[32 * 32];
    double Cl[32 * 32];
    double dv[32];
    int active[32];
    int notconv;
};

// The Gram entries this thread stages: fetched into registers first so that
// the workgroup's other loads can be issued behind them.
constexpr int kGramRegs = 32 * 32 / kThreads;
__device__ __forceinline__ void gram_fetch(gptr<const double> gram, int s, double (&v)[kGramRegs])
{
    const int ss = s * s;
#pragma unroll
    for (int q = 0; q < kGramRegs; ++q) {
        const int e = threadIdx.x + q * kThreads;
        v[q] = e < ss ? gram[e] : 0.0;
    }
}

__device__ __forceinline__ void gram_stash(const double (&v)[kGramRegs], int s, FacScratch &fs)
{
    const int ss = s * s;
#pragma unroll
    for (int q = 0; q < kGramRegs; ++q) {
        const int e = threadIdx.x + q * kThreads;
        if (e < ss) fs.A[(e / s) * (s + 1) + e % s] = v[q];
    }
}

// The calling workgroup factors the Gram it stashed in fs.A (s <= SP <= 32;
// the workgroup has synchronised since): wave 0 eliminates [G | I] into
// fs.A while the other waves run overlap(), then fs.dv = 1 / pivot (mode 0)
// or 1 / sqrt(pivot).  Every workgroup that calls this on the same Gram gets
// the same factors.
template <int SP, class F>
__device__ __forceinline__ void factor_small(int s, double rel_thr, int mode, FacScratch &fs, F overlap)
{
    static_assert(kFacThreads == kThreads, "the fused kernels factor with their own workgroup");
    if (threadIdx.x < 64) wave_eliminate<SP>(fs.A, s + 1, s, rel_thr, fs.A, fs.active);
    else overlap();
    __syncthreads();
    const int w = 2 * s;
    for (int k = threadIdx.x; k < s; k += kFacThreads)
        fs.dv[k] = !fs.active[k] ? 0.0 : (mode == 0 ? 1.0 / fs.A[k * w + k] : 1.0 / sqrt(fs.A[k * w + k]));
    __syncthreads();
}

// Factor the reduced Gram of the chip.  mode 0: delta -> M2 = delta^+, M1 = delta^+ C.
// mode 1 / 2: W^T W -> S = D^{1/2} Lunit^T, Linv = D^{-1/2} E; C <- S C;
// M3[k][j] = Linv[j][k] (Q = W S^+), M4[k][j] = S[j][k] (P = Q + P S^T);
// converged when ||C e_j|| <= th_j for every column (mode 2 is the first QR
// of the residual and is not counted as an iteration).
//
// Work layout: a blocked masked LDL^T of [G11 G12; G21 G22] with G11 the
// leading 32 x 32 block: one wavefront eliminates [G11 | I] (readlane
// broadcasts), the matrix cores form U12 = E11 G12 and the Schur complement
// G22 - U12^T D1^+ U12, one wavefront eliminates it, and the matrix cores
// assemble E21 = -E22 (U12^T D1^+) E11.  In exact arithmetic this is the
// sequential elimination (inactive pivots contribute nothing to the Schur
// complement); every pivot is tested against the same threshold on the
// largest diagonal of G.  The s x s products afterwards run on the FP64
// matrix cores too.  One workgroup per chip runs alone on its compute unit,
// so the kernel may use the whole register file (one wave per SIMD).
__global__ __launch_bounds__(kFacThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void factor_kernel(
    const ChipDev *__restrict__ cds, int s, double rel_thr, int mode)
{
    const ChipDev &cd = cds[blockIdx.x];  // one workgroup per chip
    const gptr<int> ctrl = glb(cd.ctrl);
    if (ctrl[kConverged]) return;
    const gptr<const double> __restrict__ gram = glb(static_cast<const double *>(cd.gram));
    const SmallG sm(cd.sm);
    extern __shared__ __align__(16) double lds[];
    const int ss = s * s, w = 2 * s;
    double *A = lds;       // s x 2s: [U | E]
    double *G = A + 2 * ss;  // s x s: the symmetrised Gram, then scratch
    double *Cl = G + ss;   // C
    __shared__ int active[kMaxS];
    __shared__ double dv[kMaxS];
    __shared__ double dp1[32];  // 1 / pivot of the first block (0 if inactive)
    __shared__ double gmax;
    __shared__ int notconv;
    const int tid = threadIdx.x;
    const int s1 = s < 32 ? s : 32, s2 = s - s1;
    {
        // all loads of C and of the Gram (and its transpose, which makes the
        // symmetrised entry 0.5 (G[i][j] + G[j][i]) in registers) in flight
        // before the LDS stores
        constexpr int IT = kMaxS * kMaxS / kFacThreads;
        double cv[IT], gv[IT], gt[IT];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int e = tid + i * kFacThreads;
            cv[i] = e < ss ? sm.C[e] : 0.0;
            gv[i] = e < ss ? gram[e] : 0.0;
            gt[i] = e < ss ? gram[(e % s) * s + e / s] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int e = tid + i * kFacThreads;
            if (e < ss) {
                Cl[e] = cv[i];
                G[e] = 0.5 * (gv[i] + gt[i]);
            }
        }
    }
    // structural zeros of U21 and E12 (every other entry of [U | E] is written
    // by the eliminations and products below)
    for (int e = tid; e < s2 * s1; e += kFacThreads) {
        const int i = e / s1, j = e % s1;
        A[(s1 + i) * w + j] = 0.0;
        A[j * w + s + s1 + i] = 0.0;
    }
    if (tid == 0) notconv = 0;
    __syncthreads();
    // the largest diagonal
    if (tid < 64) {
        double v = tid < s ? G[tid * s + tid] : 0.0;
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        if (tid == 0) gmax = v;
    }
    __syncthreads();
    const double gm = gmax;
    if (tid < 64) wave_eliminate<32, true>(G, s, s1, rel_thr, A, active, gm, w, s);
    __syncthreads();
    if (s2 > 0) {
        for (int k = tid; k < s1; k += kFacThreads) dp1[k] = active[k] ? 1.0 / A[k * w + k] : 0.0;
        // U12 = E11 G12 (E11[i][k] = A[i][s + k])
        small_gemm<8>(
            32, [&](int i, int k) { return A[i * w + s + k]; },
            [&](int k, int j) {
                const double v = G[k * s + s1 + j];
                return j < s2 ? v : 0.0;
            },
            [&](int i, int j, double v) {
                if (j < s2) A[i * w + s1 + j] = v;
            });
        __syncthreads();
        // Schur complement G22 -= U12^T D1^+ U12, in place
        small_gemm<8>(
            32,
            [&](int i, int k) {
                const double v = A[k * w + s1 + i] * dp1[k];
                return i < s2 ? v : 0.0;
            },
            [&](int k, int j) {
                const double v = A[k * w + s1 + j];
                return j < s2 ? v : 0.0;
            },
            [&](int i, int j, double v) {
                if (i < s2 && j < s2) G[(s1 + i) * s + s1 + j] -= v;
            });
        __syncthreads();
        if (tid < 64) wave_eliminate<32>(G + s1 * s + s1, s, s2, rel_thr, A + s1 * w + s1, active + s1, gm, w, s);
        // T1 = U12^T D1^+ E11 (s2 x s1) into the G11 block, no longer read
        // (E11 is lower triangular: k >= j)
        small_gemm<8>(
            32,
            [&](int i, int k) {
                const double v = A[k * w + s1 + i] * dp1[k];
                return i < s2 ? v : 0.0;
            },
            [&](int k, int j) { return A[k * w + s + j]; },
            [&](int i, int j, double v) {
                if (i < s2) G[i * s + j] = v;
            },
            [](int, int bj) { return 4 * bj; });
        __syncthreads();
        // E21 = -E22 T1 (E22[i][k] = A[s1 + i][s + s1 + k])
        small_gemm<8>(
            32,
            [&](int i, int k) {
                const double v = A[(s1 + i) * w + s + s1 + k];
                return (i < s2 && k < s2) ? v : 0.0;
            },
            [&](int k, int j) {
                const double v = G[k * s + j];
                return k < s2 ? v : 0.0;
            },
            [&](int i, int j, double v) {
                if (i < s2) A[(s1 + i) * w + s + j] = -v;
            });
    }
    __syncthreads();
    for (int k = tid; k < s; k += kFacThreads)
        dv[k] = !active[k] ? 0.0 : (mode == 0 ? 1.0 / A[k * w + k] : 1.0 / sqrt(A[k * w + k]));
    __syncthreads();
    int inactive = 0;
    for (int k = 0; k < s; ++k) inactive += active[k] ? 0 : 1;
    if (mode == 0) {
        // delta^+ = E^T diag(dv) E (E = right half, lower triangular: only
        // k >= max(i, j) contributes); M2 = delta^+, M1 = delta^+ C
        small_gemm<kMaxS / 4>(
            s, [&](int i, int k) { return A[k * w + s + i]; }, [&](int k, int j) { return dv[k] * A[k * w + s + j]; },
            [&](int i, int j, double v) {
                G[i * s + j] = v;
                sm.M2[i * s + j] = v;
                sm.M2f[i * s + j] = static_cast<float>(v);
            },
            [](int bi, int bj) { return 4 * (bi > bj ? bi : bj); });
        __syncthreads();
        small_gemm<kMaxS / 4>(
            s, [&](int i, int k) { return G[i * s + k]; }, [&](int k, int j) { return Cl[k * s + j]; },
            [&](int i, int j, double v) {
                sm.M1[i * s + j] = v;
                sm.M1f[i * s + j] = static_cast<float>(v);
            });
        return;
    }
    // Cn = S C into G, S[i][k] = U[i][k] dv[i] (k >= i)
    small_gemm<kMaxS / 4>(
        s,
        [&](int i, int k) {
            const double v = A[i * w + k] * dv[i];
            return k >= i ? v : 0.0;
        },
        [&](int k, int j) { return Cl[k * s + j]; }, [&](int i, int j, double v) { G[i * s + j] = v; },
        [](int bi, int) { return 4 * bi; });
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

// ------------------------------------------------------------------ block updates

// Stage NM s x s matrices (row-major, ld s) as padded SP x MST tiles of T in
// LDS; entries outside s x s are zero and neg[q] negates matrix q.  The
// loads of every matrix are issued in groups before their LDS stores, so a
// workgroup pays a few memory latencies here, not one per element it stages.
template <class T, int SP, int MST, int NM>
__device__ inline void stage_small(T *const (&dst)[NM], const gptr<const T> (&src)[NM], int s, const bool (&neg)[NM])
{
    constexpr int IT = (SP * MST + kThreads - 1) / kThreads;
    constexpr int CH = IT < 6 ? IT : 6;
    for (int i0 = 0; i0 < IT; i0 += CH) {
        T v[NM][CH];
#pragma unroll
        for (int q = 0; q < NM; ++q)
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int e = threadIdx.x + (i0 + i) * kThreads;
                const int k = e / MST, j = e % MST;
                v[q][i] = (i0 + i < IT && e < SP * MST && k < s && j < s) ? src[q][k * s + j] : T(0);
            }
#pragma unroll
        for (int q = 0; q < NM; ++q)
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int e = threadIdx.x + (i0 + i) * kThreads;
                if (i0 + i < IT && e < SP * MST) dst[q][e] = neg[q] ? -v[q][i] : v[q][i];
            }
    }
}

// stage_small split in two for one matrix: fetch its entries of the padded
// SP x MST tile into registers (so that later loads can be issued behind
// them), then store them to LDS.
template <int SP, int MST> constexpr int small_regs() { return (SP * MST + kThreads - 1) / kThreads; }

template <class T, int SP, int MST>
__device__ __forceinline__ void small_fetch(gptr<const T> src, int s, T (&v)[small_regs<SP, MST>()])
{
#pragma unroll
    for (int i = 0; i < small_regs<SP, MST>(); ++i) {
        const int e = threadIdx.x + i * kThreads;
        const int k = e / MST, j = e % MST;
        v[i] = (e < SP * MST && k < s && j < s) ? src[k * s + j] : T(0);
    }
}

template <class T, int SP, int MST>
__device__ __forceinline__ void small_stash(T *dst, const T (&v)[small_regs<SP, MST>()], bool neg)
{
#pragma unroll
    for (int i = 0; i < small_regs<SP, MST>(); ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < SP * MST) dst[e] = neg ? -v[i] : v[i];
    }
}

// W <- W M3 - AP M2 (the previous step's Q = W S^+ formed on the fly, matrix
// cores in the storage precision) and the W^T W partials from the same
// registers.  With init != 0, W holds the residual and only its Gram is
// formed.  W is updated in place: each wave reads a 16-row block of every
// column before it writes that block.
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void update_w_kernel(const ChipDev *__restrict__ cds,
                                                            const uint16_t *__restrict__ tab, int s, int init)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (glb(cd.ctrl)[kConverged]) return;
    using V = typename MF<T>::V;
    constexpr bool kF64 = MF<T>::kF64;
    constexpr int KS = 4 * NB;  // k steps of 4 over the padded width 16 NB
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    __shared__ T M3s[SP * MST];
    __shared__ T M2s[SP * MST];  // -M2
    __shared__ double lds[kMaxS * kMaxS];
    const bool f64 = sizeof(T) == 8;
    if (!init) {
        T *const dst[2] = {M3s, M2s};
        const gptr<const T> src[2] = {glb(f64 ? reinterpret_cast<const T *>(cd.sm.M3) : reinterpret_cast<const T *>(cd.sm.M3f)),
                                      glb(f64 ? reinterpret_cast<const T *>(cd.sm.M2) : reinterpret_cast<const T *>(cd.sm.M2f))};
        const bool neg[2] = {false, true};
        stage_small<T, SP, MST, 2>(dst, src, s, neg);
        __syncthreads();
    }
    const gptr<T> __restrict__ W = glb(static_cast<T *>(cd.W));
    const gptr<const T> __restrict__ AP = glb(static_cast<const T *>(cd.AP));
    const int64_t ldw = cd.ldw;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    d4 g[NB * (NB + 1) / 2];
#pragma unroll
    for (int q = 0; q < NB * (NB + 1) / 2; ++q) g[q] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t ntiles = ldw / kTileRows;
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t r0 = tile * kTileRows + wave * 64 + rb * 16;
            V wv[NB];
            if (init) {
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        wv[jb][r] = colj < s ? W[colj * ldw + r0 + mfma_row<kF64>(lg, r)] : T(0);
                }
            } else {
                T wa[KS], aa[KS];
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const int col = 4 * t + lg;
                    wa[t] = col < s ? W[col * ldw + r0 + li] : T(0);
                    aa[t] = col < s ? AP[col * ldw + r0 + li] : T(0);
                }
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
                    V acc;
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] = T(0);
                    // S^+ is upper triangular: no k steps below the column block
#pragma unroll
                    for (int t = 0; t < 4 * (jb + 1); ++t) acc = MF<T>::mma(wa[t], M3s[(4 * t + lg) * MST + colj], acc);
#pragma unroll
                    for (int t = 0; t < KS; ++t) acc = MF<T>::mma(aa[t], M2s[(4 * t + lg) * MST + colj], acc);
                    wv[jb] = acc;
                }
                // every lane has read its rows of W: write the new block
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
                    if (colj < s) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) W[colj * ldw + r0 + mfma_row<kF64>(lg, r)] = wv[jb][r];
                    }
                }
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
    static_assert(kMaxS * kMaxS >= publish_lds<kThreads>(4), "publish_partial LDS");
    publish_partial<NB, true>(g, s, lds, glb(cd.parts) + static_cast<size_t>(local) * s * s);
}

// The W update in FP32 for s > 32 (blocks streamed from HBM): a wave takes
// 32 rows at a time as two interleaved 16-row matrix-core blocks (block q
// holds rows 2 i + q), so that one 8-byte load gives a lane its operand in
// both blocks and 16 lanes read a whole 128-byte line of a column; result
// register r of the two blocks holds 2 consecutive rows (8 g + 2 r, + 1 for
// lane group g), one 8-byte store.  The W^T W partial is shared out over the
// waves: the 128 new rows of the four waves are staged in LDS (row stride of
// 80 floats, so the four lane groups of a matrix-core read fall on disjoint
// banks) and each wave accumulates whole upper 16 x 16 blocks of the Gram
// over all of them on the FP64 matrix cores (NB (NB + 1) / 2 blocks: two per
// wave for s <= 64, one for s <= 48, and the last two blocks split by rows
// between pairs of waves).  Each wave then holds 3 or 2 accumulator blocks
// instead of all of them, which keeps the kernel at two waves per SIMD.
template <int NB>
__global__ __launch_bounds__(kThreads) void update_w_rows2_kernel(const ChipDev *__restrict__ cds,
                                                                     const uint16_t *__restrict__ tab, int s, int init)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (glb(cd.ctrl)[kConverged]) return;
    constexpr int KS = 4 * NB;
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    constexpr int NBLK = NB * (NB + 1) / 2;
    static_assert(NBLK % 4 == 2, "the Gram blocks split as whole blocks per wave plus two shared ones");
    constexpr int FB = NBLK / 4;  // whole Gram blocks per wave
    constexpr int SR = 4 * 32;    // rows staged per half tile (four waves x 32)
    constexpr int WST = 80;       // row stride of the staged rows, floats
    static_assert(SP <= WST, "staged row width");
    __shared__ float M3s[SP * MST];
    __shared__ float M2s[SP * MST];  // -M2
    __shared__ __align__(16) float Wst[SR * WST];
    if (!init) {
        float *const dst[2] = {M3s, M2s};
        const gptr<const float> src[2] = {glb(static_cast<const float *>(cd.sm.M3f)),
                                          glb(static_cast<const float *>(cd.sm.M2f))};
        const bool neg[2] = {false, true};
        stage_small<float, SP, MST, 2>(dst, src, s, neg);
        __syncthreads();
    }
    const gptr<float> __restrict__ W = glb(static_cast<float *>(cd.W));
    const gptr<const float> __restrict__ AP = glb(static_cast<const float *>(cd.AP));
    const int64_t ldw = cd.ldw;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const f2 zero = {0.f, 0.f};
    auto ld8 = [](gptr<const float> p) { return *reinterpret_cast<gptr<const f2>>(p); };
    // this wave's Gram blocks: whole blocks wave + 4 f (f < FB), then half
    // of block 4 FB + wave / 2 (rows 64 (wave % 2) .. + 64 of the stage)
    int ga[FB + 1], gb[FB + 1];
#pragma unroll
    for (int f = 0; f < FB; ++f) gram_block<NB, true>(wave + 4 * f, ga[f], gb[f]);
    gram_block<NB, true>(4 * FB + (wave >> 1), ga[FB], gb[FB]);
    const int hk0 = (wave & 1) * (SR / 2);
    d4 g[FB + 1];
#pragma unroll
    for (int q = 0; q <= FB; ++q) g[q] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t ntiles = ldw / kTileRows;
    // stage one unit's new rows (columns s .. SP are zero: their operands
    // were), then W^T W over the staged rows (row k0 + lg is the k slot of
    // lane group lg)
    auto stage_gram = [&](const f4 (&wv)[NB][2]) {
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Wst[(wave * 32 + 8 * lg + 2 * r + q) * WST + jb * 16 + li] = wv[jb][q][r];
        __syncthreads();
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const float *pa = Wst + lg * WST + ga[f] * 16 + li, *pb = Wst + lg * WST + gb[f] * 16 + li;
#pragma unroll 8
            for (int k0 = 0; k0 < SR; k0 += 4)
                g[f] = mma64(static_cast<double>(pa[k0 * WST]), static_cast<double>(pb[k0 * WST]), g[f]);
        }
        {
            const float *pa = Wst + (hk0 + lg) * WST + ga[FB] * 16 + li;
            const float *pb = Wst + (hk0 + lg) * WST + gb[FB] * 16 + li;
#pragma unroll 8
            for (int k0 = 0; k0 < SR / 2; k0 += 4)
                g[FB] = mma64(static_cast<double>(pa[k0 * WST]), static_cast<double>(pb[k0 * WST]), g[FB]);
        }
        __syncthreads();  // the next unit overwrites the stage
    };
    if (init) {
        for (int64_t tile = local; tile < ntiles; tile += wgs)
            for (int h = 0; h < 2; ++h) {
                const int64_t r0 = tile * kTileRows + wave * 64 + 32 * h;
                f4 wv[NB][2];
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const f2 v = colj < s ? ld8(gptr<const float>(W) + colj * ldw + r0 + 8 * lg + 2 * r) : zero;
                        wv[jb][0][r] = v[0];
                        wv[jb][1][r] = v[1];
                    }
                }
                stage_gram(wv);
            }
    } else if (local < ntiles) {
        // W M3 + AP (-M2) in one pass over the k steps: the W and AP rows
        // of each step stream through a ring of kDepth register slots,
        // refilled kDepth steps ahead; the last steps of a 32-row unit fetch
        // the first ones of the next, so those loads fly during this unit's
        // stores, stage and Gram products (8 slots measured 4 % faster than 4
        // at s = 64)
        constexpr int kDepth = NB == 4 ? 8 : 4;
        static_assert(KS % kDepth == 0, "a unit holds whole ring turns");
        f2 rw[kDepth], rp[kDepth];
        auto fetch = [&](int64_t r0, int t, f2 &xw, f2 &xp) {
            const int col = 4 * t + lg;
            const int64_t a = col * ldw + r0 + 2 * li;
            xw = col < s ? ld8(gptr<const float>(W) + a) : zero;
            xp = col < s ? ld8(AP + a) : zero;
        };
        const int64_t u_first = local * kTileRows + wave * 64;
#pragma unroll
        for (int d = 0; d < kDepth; ++d) fetch(u_first, d, rw[d], rp[d]);
        for (int64_t tile = local; tile < ntiles; tile += wgs)
            for (int h = 0; h < 2; ++h) {
                const int64_t r0 = tile * kTileRows + wave * 64 + 32 * h;
                const bool has_next = h == 0 || tile + wgs < ntiles;
                const int64_t r0n = h == 0 ? r0 + 32 : (tile + wgs) * kTileRows + wave * 64;
                f4 wv[NB][2];
#pragma unroll
                for (int jb = 0; jb < NB; ++jb)
#pragma unroll
                    for (int q = 0; q < 2; ++q) wv[jb][q] = f4{0.f, 0.f, 0.f, 0.f};
                // the small-matrix entries of step t + 1 are read during
                // step t; the empty asm keeps the compiler from hoisting all
                // of them (unit-invariant) into registers for the whole loop
                int mb = lg * MST + li;
                float m3[2][NB], m2[2][NB];
                auto read_m = [&](int t, int slot) {
                    const int tb = t / 4;
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) {
                        const int o = mb + 4 * t * MST + jb * 16;
                        m3[slot][jb] = jb >= tb ? M3s[o] : 0.f;
                        m2[slot][jb] = M2s[o];
                    }
                };
                asm volatile("" : "+v"(mb));
                read_m(0, 0);
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const int tb = t / 4, cs = t & 1;
                    asm volatile("" : "+v"(mb));
                    if (t + 1 < KS) read_m(t + 1, cs ^ 1);
                    const f2 xw = rw[t % kDepth], xp = rp[t % kDepth];
                    // M3 = S^+ is upper triangular: column block jb takes
                    // its k steps only for tb <= jb
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) {
                        if (jb >= tb) {
#pragma unroll
                            for (int q = 0; q < 2; ++q) wv[jb][q] = MF<float>::mma(xw[q], m3[cs][jb], wv[jb][q]);
                        }
#pragma unroll
                        for (int q = 0; q < 2; ++q) wv[jb][q] = MF<float>::mma(xp[q], m2[cs][jb], wv[jb][q]);
                    }
                    const int tn = t + kDepth;
                    if (tn < KS) fetch(r0, tn, rw[t % kDepth], rp[t % kDepth]);
                    else if (has_next) fetch(r0n, tn - KS, rw[t % kDepth], rp[t % kDepth]);
                }
                // every lane has read its rows of W: write the new rows
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
                    if (colj < s) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const f2 v = {wv[jb][0][r], wv[jb][1][r]};
                            *reinterpret_cast<gptr<f2>>(W + colj * ldw + r0 + 8 * lg + 2 * r) = v;
                        }
                    }
                }
                stage_gram(wv);
            }
    }
    // publish: whole blocks by their wave; the shared blocks summed through LDS
    const gptr<double> out = glb(cd.parts) + static_cast<size_t>(local) * s * s;
    auto put = [&](int a, int b, const d4 &v) {
        const int j = b * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = a * 16 + mfma_row<true>(lg, r);
            if (i < s && j < s) {
                out[i * s + j] = v[r];
                if (a != b) out[j * s + i] = v[r];
            }
        }
    };
#pragma unroll
    for (int f = 0; f < FB; ++f) put(ga[f], gb[f], g[f]);
    double *xs = reinterpret_cast<double *>(Wst);
    if (wave & 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) xs[((wave >> 1) * 4 + r) * 64 + lane] = g[FB][r];
    }
    __syncthreads();
    if (!(wave & 1)) {
        d4 v = g[FB];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] += xs[((wave >> 1) * 4 + r) * 64 + lane];
        put(ga[FB], gb[FB], v);
    }
}

// D += P M1 ;  P = W M3 + P M4   (matrix cores, storage precision; Q = W M3)
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void update_dqp_kernel(const ChipDev *__restrict__ cds,
                                                              const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (glb(cd.ctrl)[kStop]) return;
    using V = typename MF<T>::V;
    constexpr bool kF64 = MF<T>::kF64;
    constexpr int KS = 4 * NB;
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    extern __shared__ __align__(16) double dlds[];
    T *M1 = reinterpret_cast<T *>(dlds);
    T *M3 = M1 + SP * MST;
    T *M4 = M3 + SP * MST;
    const bool f64 = sizeof(T) == 8;
    {
        T *const dst[3] = {M1, M3, M4};
        const gptr<const T> src[3] = {
            glb(f64 ? reinterpret_cast<const T *>(cd.sm.M1) : reinterpret_cast<const T *>(cd.sm.M1f)),
            glb(f64 ? reinterpret_cast<const T *>(cd.sm.M3) : reinterpret_cast<const T *>(cd.sm.M3f)),
            glb(f64 ? reinterpret_cast<const T *>(cd.sm.M4) : reinterpret_cast<const T *>(cd.sm.M4f))};
        const bool neg[3] = {false, false, false};
        stage_small<T, SP, MST, 3>(dst, src, s, neg);
    }
    __syncthreads();
    const gptr<T> __restrict__ D = glb(static_cast<T *>(cd.Dv));
    const gptr<T> __restrict__ P = glb(static_cast<T *>(cd.P));
    const gptr<const T> __restrict__ W = glb(static_cast<const T *>(cd.W));
    const int64_t ldw = cd.ldw;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t ntiles = ldw / kTileRows;
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t r0 = tile * kTileRows + wave * 64 + rb * 16;
            T pa[KS], wa[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int col = 4 * t + lg;
                pa[t] = col < s ? P[col * ldw + r0 + li] : T(0);
                wa[t] = col < s ? W[col * ldw + r0 + li] : T(0);
            }
            // pa holds this wave's rows of every column of P, so the new rows
            // can be written column block by column block (a loop for s > 32,
            // which keeps the small-matrix reads of one block in registers)
#pragma unroll(NB > 2 ? 1 : NB)
            for (int jb = 0; jb < NB; ++jb) {
                const int colj = jb * 16 + li;
                V ad, ap;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ad[r] = colj < s ? D[colj * ldw + r0 + mfma_row<kF64>(lg, r)] : T(0);
                    ap[r] = T(0);
                }
                // S^+ upper, S^T lower triangular: only their nonzero 16-row
                // blocks (jb is uniform: the guards are scalar branches)
#pragma unroll
                for (int t = 0; t < KS; ++t) {
                    const int k = 4 * t + lg;
                    ad = MF<T>::mma(pa[t], M1[k * MST + colj], ad);
                    if (t < 4 * (jb + 1)) ap = MF<T>::mma(wa[t], M3[k * MST + colj], ap);
                }
#pragma unroll
                for (int t = 0; t < KS; ++t)
                    if (t >= 4 * jb) ap = MF<T>::mma(pa[t], M4[(4 * t + lg) * MST + colj], ap);
                if (colj < s) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t idx = colj * ldw + r0 + mfma_row<kF64>(lg, r);
                        D[idx] = ad[r];
                        P[idx] = ap[r];
                    }
                }
            }
        }
    }
}

// The same update in FP32 for s > 32, where the N x s blocks no longer fit
// the Infinity Cache and come from HBM.  A wave takes 64 rows as four
// interleaved 16-row blocks (block q holds rows 4 i + q, i = 0..15), so that
// one 16-byte load gives a lane its operand in all four blocks and 16 lanes
// read 256 contiguous bytes of a column.  The products are formed
// transposed, (P M)^T = M^T P^T: the small matrix is the matrix-core A
// operand and the rows of P the B operand, so that result register r of
// lane (i, g) is column 16 jb + 4 g + r at row 4 i + q; the four blocks then
// give a lane 4 consecutive rows of one column, and 16 lanes write (and
// read, for D) 256 contiguous bytes of it with one 16-byte access each.  In
// the untransposed form each such access touched 16 columns in 16-byte
// pieces, and the kernel ran 30 % slower.
//
// The wave keeps all 2 s new columns of its rows in accumulators and streams
// the k steps of P and W through a ring of kDepth register slots, each
// refilled kDepth steps ahead (the last steps of a tile fetch the first ones
// of the next), so that the loads overlap the matrix-core work instead of
// preceding it.  D is not the accumulators' start value: column block jb of
// D is loaded at step 3 jb and added in at step 3 jb + 3, which keeps its
// load latency off the chain too.
template <int NB, int kDepth = 4>
__global__ __launch_bounds__(kThreads) void update_dqp_rows4_kernel(const ChipDev *__restrict__ cds,
                                                                    const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (glb(cd.ctrl)[kStop]) return;
    constexpr int KS = 4 * NB;
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    static_assert(KS % kDepth == 0 && 3 * NB < KS, "a tile holds whole ring turns and the D schedule");
    extern __shared__ __align__(16) double dlds[];
    float *M1 = reinterpret_cast<float *>(dlds);
    float *M3 = M1 + SP * MST;
    float *M4 = M3 + SP * MST;
    {
        float *const dst[3] = {M1, M3, M4};
        const gptr<const float> src[3] = {glb(static_cast<const float *>(cd.sm.M1f)),
                                          glb(static_cast<const float *>(cd.sm.M3f)),
                                          glb(static_cast<const float *>(cd.sm.M4f))};
        const bool neg[3] = {false, false, false};
        stage_small<float, SP, MST, 3>(dst, src, s, neg);
    }
    __syncthreads();
    const gptr<float> __restrict__ D = glb(static_cast<float *>(cd.Dv));
    const gptr<float> __restrict__ P = glb(static_cast<float *>(cd.P));
    const gptr<const float> __restrict__ W = glb(static_cast<const float *>(cd.W));
    const int64_t ldw = cd.ldw;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t ntiles = ldw / kTileRows;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    if (local >= ntiles) return;
    f4 pr[kDepth], wr[kDepth];
    auto fetch = [&](int64_t tile, int t, f4 &pv, f4 &wv) {
        const int col = 4 * t + lg;
        const int64_t a = col * ldw + tile * kTileRows + wave * 64 + 4 * li;
        pv = col < s ? ld16(gptr<const float>(P) + a) : zero;
        wv = col < s ? ld16(W + a) : zero;
    };
#pragma unroll
    for (int d = 0; d < kDepth; ++d) fetch(local, d, pr[d], wr[d]);
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        const int64_t r0 = tile * kTileRows + wave * 64;
        const int64_t nxt = tile + wgs;
        f4 ad[NB][4], ap[NB][4], dv[4];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int q = 0; q < 4; ++q) ad[jb][q] = ap[jb][q] = zero;
        // the small-matrix entries of step t + 1 are read during step t; the
        // empty asm re-defines their LDS index every step, which keeps the
        // compiler from hoisting all of them (they do not change from tile
        // to tile) into registers for the whole loop
        int mb = lg * MST + li;
        float m1[2][NB], m3[2][NB], m4[2][NB];
        auto read_m = [&](int t, int slot) {
            const int tb = t / 4;
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int o = mb + 4 * t * MST + jb * 16;
                m1[slot][jb] = M1[o];
                m3[slot][jb] = jb >= tb ? M3[o] : 0.f;
                m4[slot][jb] = jb <= tb ? M4[o] : 0.f;
            }
        };
        asm volatile("" : "+v"(mb));
        read_m(0, 0);
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const int tb = t / 4;
            const int cs = t & 1;
            asm volatile("" : "+v"(mb));
            if (t + 1 < KS) read_m(t + 1, cs ^ 1);
            const f4 pa = pr[t % kDepth], wa = wr[t % kDepth];
            // M3 = S^+ is upper and M4 = S^T lower triangular: column block
            // jb takes M3's k steps only for tb <= jb and M4's only for tb >= jb
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
#pragma unroll
                for (int q = 0; q < 4; ++q) ad[jb][q] = MF<float>::mma(m1[cs][jb], pa[q], ad[jb][q]);
                if (jb >= tb) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) ap[jb][q] = MF<float>::mma(m3[cs][jb], wa[q], ap[jb][q]);
                }
                if (jb <= tb) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) ap[jb][q] = MF<float>::mma(m4[cs][jb], pa[q], ap[jb][q]);
                }
            }
            if (t % 3 == 0 && t / 3 >= 1 && t / 3 <= NB) {
                const int jb = t / 3 - 1;
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ad[jb][q][r] += dv[r][q];
            }
            if (t % 3 == 0 && t / 3 < NB) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = (t / 3) * 16 + 4 * lg + r;
                    dv[r] = c < s ? ld16(gptr<const float>(D) + c * ldw + r0 + 4 * li) : zero;
                }
            }
            const int tn = t + kDepth;
            if (tn < KS) fetch(tile, tn, pr[t % kDepth], wr[t % kDepth]);
            else if (nxt < ntiles) fetch(nxt, tn - KS, pr[t % kDepth], wr[t % kDepth]);
        }
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = jb * 16 + 4 * lg + r;
                if (c < s) {
                    const int64_t idx = c * ldw + r0 + 4 * li;
                    const f4 dn = {ad[jb][0][r], ad[jb][1][r], ad[jb][2][r], ad[jb][3][r]};
                    const f4 pn = {ap[jb][0][r], ap[jb][1][r], ap[jb][2][r], ap[jb][3][r]};
                    *reinterpret_cast<gptr<f4>>(D + idx) = dn;
                    *reinterpret_cast<gptr<f4>>(P + idx) = pn;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ fused factorisation + update (s <= 32)
//
// For s <= 32 the two s x s factorisations of an iteration run inside the
// kernels that consume them: every workgroup factors the reduced Gram
// itself (one wavefront, identical results in every workgroup), which
// removes two launches and their gaps from each iteration.  Workgroup 0 of
// the chip also publishes what later kernels need (M1 for the D update, C,
// M3, the control words).
//
// The factorisation's latency is partly hidden: the Gram and the small
// matrices are fetched first and staged in LDS, then, while wave 0
// eliminates, waves 1..3 load their first row blocks and do the part of
// their update that does not depend on the new factors (W S^+ here, D +=
// P M1 in update_dqp); wave 0 loads its rows and does its part in the row
// loop, so the eliminating wave holds no row data.

// 16-row blocks per wave held in registers at once by the fused kernels
// (FP64 holds fewer, to keep two waves per SIMD).
template <class T, bool kW> constexpr int fused_rows() { return sizeof(T) == 4 ? 4 : (kW ? 1 : 2); }

// W <- W S^+ - AP delta^+ with delta^+ factored here (see update_w_kernel).
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void update_w_fused_kernel(const ChipDev *__restrict__ cds,
                                                                  const uint16_t *__restrict__ tab, int s,
                                                                  double rel_thr)
{
    static_assert(NB <= 2, "fused factorisation is for s <= 32");
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    // the control word is tested after the Gram and the small matrices are
    // requested, so that their loads overlap its latency
    const int stop = glb(cd.ctrl)[kConverged];
    using V = typename MF<T>::V;
    constexpr bool kF64 = MF<T>::kF64;
    constexpr int KS = 4 * NB;
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    constexpr int PRE = fused_rows<T, true>();
    constexpr int NG = 4 / PRE;
    __shared__ T M3s[SP * MST];
    __shared__ T M2s[SP * MST];  // -delta^+
    __shared__ FacScratch fs;
    const bool f64 = sizeof(T) == 8;
    const SmallG sm(cd.sm);
    const gptr<T> __restrict__ W = glb(static_cast<T *>(cd.W));
    const gptr<const T> __restrict__ AP = glb(static_cast<const T *>(cd.AP));
    const int64_t ldw = cd.ldw;
    const int64_t ntiles = ldw / kTileRows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    T wa[PRE][KS], aa[PRE][KS];
    V wm[PRE][NB];  // W S^+ of the held row blocks
    auto load = [&](int64_t tile, int gi) {
#pragma unroll
        for (int p = 0; p < PRE; ++p) {
            const int64_t r0 = tile * kTileRows + wave * 64 + (gi * PRE + p) * 16;
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int col = 4 * t + lg;
                wa[p][t] = col < s ? W[col * ldw + r0 + li] : T(0);
                aa[p][t] = col < s ? AP[col * ldw + r0 + li] : T(0);
            }
        }
    };
    auto part_w = [&]() {
#pragma unroll
        for (int p = 0; p < PRE; ++p)
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int colj = jb * 16 + li;
                V acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = T(0);
                // S^+ is upper triangular: no k steps below the column block
#pragma unroll
                for (int t = 0; t < 4 * (jb + 1); ++t) acc = MF<T>::mma(wa[p][t], M3s[(4 * t + lg) * MST + colj], acc);
                wm[p][jb] = acc;
            }
    };
    double gv[kGramRegs], cv[kGramRegs];
    T mv[small_regs<SP, MST>()];
    gram_fetch(glb(static_cast<const double *>(cd.gram)), s, gv);
    small_fetch<T, SP, MST>(glb(f64 ? reinterpret_cast<const T *>(cd.sm.M3) : reinterpret_cast<const T *>(cd.sm.M3f)),
                            s, mv);
    if (local == 0) gram_fetch(sm.C, s, cv);
    if (stop) return;
    const bool first = local < ntiles;
    small_stash<T, SP, MST>(M3s, mv, false);
    for (int e = threadIdx.x; e < SP * MST; e += kThreads) M2s[e] = T(0);
    gram_stash(gv, s, fs);
    __syncthreads();
    factor_small<SP>(s, rel_thr, 0, fs, [&] {
        if (first) {
            load(local, 0);
            part_w();
        }
    });
    const int w = 2 * s;
    // delta^+ = E^T diag(dv) E (E = right half of the eliminated [G | I],
    // lower triangular: only k >= max(i, j) contributes)
    small_gemm<4 * NB>(
        s, [&](int i, int k) { return fs.A[k * w + s + i]; }, [&](int k, int j) { return fs.dv[k] * fs.A[k * w + s + j]; },
        [&](int i, int j, double v) {
            M2s[i * MST + j] = static_cast<T>(-v);
            fs.G[i * s + j] = v;
        },
        [](int bi, int bj) { return 4 * (bi > bj ? bi : bj); });
    __syncthreads();
    if (local == 0) {
        // M1 = delta^+ C for this step's update of D
#pragma unroll
        for (int q = 0; q < kGramRegs; ++q)
            if (threadIdx.x + q * kThreads < s * s) fs.Cl[threadIdx.x + q * kThreads] = cv[q];
        __syncthreads();
        small_gemm<4 * NB>(
            s, [&](int i, int k) { return fs.G[i * s + k]; }, [&](int k, int j) { return fs.Cl[k * s + j]; },
            [&](int i, int j, double v) {
                sm.M1[i * s + j] = v;
                sm.M1f[i * s + j] = static_cast<float>(v);
            });
        __syncthreads();
    }
    d4 g[NB * (NB + 1) / 2];
#pragma unroll
    for (int q = 0; q < NB * (NB + 1) / 2; ++q) g[q] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            if (tile != local || gi != 0 || wave == 0) {
                load(tile, gi);
                part_w();
            }
#pragma unroll
            for (int p = 0; p < PRE; ++p) {
                const int64_t r0 = tile * kTileRows + wave * 64 + (gi * PRE + p) * 16;
                V wv[NB];
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
                    V acc = wm[p][jb];
#pragma unroll
                    for (int t = 0; t < KS; ++t) acc = MF<T>::mma(aa[p][t], M2s[(4 * t + lg) * MST + colj], acc);
                    wv[jb] = acc;
                }
                // this wave loaded these rows of W before: write the new block
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
                    if (colj < s) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) W[colj * ldw + r0 + mfma_row<kF64>(lg, r)] = wv[jb][r];
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int ab = 0; ab < NB; ++ab)
#pragma unroll
                        for (int bb = ab; bb < NB; ++bb)
                            g[ublock<NB>(ab, bb)] = mma64(static_cast<double>(wv[ab][r]),
                                                          static_cast<double>(wv[bb][r]), g[ublock<NB>(ab, bb)]);
            }
        }
    }
    // the factor scratch is dead here: it holds the partial's reduction
    static_assert(sizeof(FacScratch) >= sizeof(double) * publish_lds<kThreads>(3), "publish_partial LDS");
    publish_partial<NB, true>(g, s, reinterpret_cast<double *>(&fs), glb(cd.parts) + static_cast<size_t>(local) * s * s);
}

// D += P M1; P = W S^+ + P S^T with W^T W = S^T S factored here (mode 1, or
// 2 for the first QR of an inner solve, which is not counted as an
// iteration); workgroup 0 updates C = S C, tests convergence on it and
// publishes S^+ for the next step.
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void update_dqp_fused_kernel(const ChipDev *__restrict__ cds,
                                                                    const uint16_t *__restrict__ tab, int s,
                                                                    double rel_thr, int mode)
{
    static_assert(NB <= 2, "fused factorisation is for s <= 32");
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    const gptr<int> ctrl = glb(cd.ctrl);
    // the control word is tested after the Gram and the small matrices are
    // requested, so that their loads overlap its latency
    const int stop = ctrl[kStop];
    using V = typename MF<T>::V;
    constexpr bool kF64 = MF<T>::kF64;
    constexpr int KS = 4 * NB;
    constexpr int SP = 16 * NB;
    constexpr int MST = SP + 1;
    constexpr int PRE = fused_rows<T, false>();
    constexpr int NG = 4 / PRE;
    __shared__ T M1[SP * MST];
    __shared__ T M3[SP * MST];
    __shared__ T M4[SP * MST];
    __shared__ FacScratch fs;
    const bool f64 = sizeof(T) == 8;
    const SmallG sm(cd.sm);
    const gptr<T> __restrict__ D = glb(static_cast<T *>(cd.Dv));
    const gptr<T> __restrict__ P = glb(static_cast<T *>(cd.P));
    const gptr<const T> __restrict__ W = glb(static_cast<const T *>(cd.W));
    const int64_t ldw = cd.ldw;
    const int64_t ntiles = ldw / kTileRows;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    T pa[PRE][KS], wa[PRE][KS], dd[PRE][NB][4];
    auto load = [&](int64_t tile, int gi) {
#pragma unroll
        for (int p = 0; p < PRE; ++p) {
            const int64_t r0 = tile * kTileRows + wave * 64 + (gi * PRE + p) * 16;
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int col = 4 * t + lg;
                pa[p][t] = col < s ? P[col * ldw + r0 + li] : T(0);
                wa[p][t] = col < s ? W[col * ldw + r0 + li] : T(0);
            }
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int colj = jb * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    dd[p][jb][r] = colj < s ? D[colj * ldw + r0 + mfma_row<kF64>(lg, r)] : T(0);
            }
        }
    };
    // D += P M1 for the held row blocks (independent of this step's factors)
    auto part_d = [&](int64_t tile, int gi) {
#pragma unroll
        for (int p = 0; p < PRE; ++p) {
            const int64_t r0 = tile * kTileRows + wave * 64 + (gi * PRE + p) * 16;
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const int colj = jb * 16 + li;
                V ad;
#pragma unroll
                for (int r = 0; r < 4; ++r) ad[r] = dd[p][jb][r];
#pragma unroll
                for (int t = 0; t < KS; ++t) ad = MF<T>::mma(pa[p][t], M1[(4 * t + lg) * MST + colj], ad);
                if (colj < s) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) D[colj * ldw + r0 + mfma_row<kF64>(lg, r)] = ad[r];
                }
            }
        }
    };
    double gv[kGramRegs], cv[kGramRegs];
    T mv[small_regs<SP, MST>()];
    gram_fetch(glb(static_cast<const double *>(cd.gram)), s, gv);
    small_fetch<T, SP, MST>(glb(f64 ? reinterpret_cast<const T *>(cd.sm.M1) : reinterpret_cast<const T *>(cd.sm.M1f)),
                            s, mv);
    int iters = 0;
    if (local == 0) {
        gram_fetch(sm.C, s, cv);
        iters = ctrl[kIters];
    }
    if (stop) return;
    const bool first = local < ntiles;
    small_stash<T, SP, MST>(M1, mv, false);
    gram_stash(gv, s, fs);
    __syncthreads();
    factor_small<SP>(s, rel_thr, mode, fs, [&] {
        if (first) {
            load(local, 0);
            part_d(local, 0);
        }
    });
    const int w = 2 * s;
    // M3[k][j] = S^+[k][j] = E[j][k] dv[j] (k <= j);  M4[k][j] = S[j][k] = U[j][k] dv[j] (k >= j)
    for (int e = threadIdx.x; e < SP * MST; e += kThreads) {
        const int k = e / MST, j = e % MST;
        const bool in = k < s && j < s;
        const double m3 = (in && k <= j) ? fs.A[j * w + s + k] * fs.dv[j] : 0.0;
        const double m4 = (in && k >= j) ? fs.A[j * w + k] * fs.dv[j] : 0.0;
        M3[e] = static_cast<T>(m3);
        M4[e] = static_cast<T>(m4);
        if (local == 0 && in) {
            sm.M3[k * s + j] = m3;
            sm.M3f[k * s + j] = static_cast<float>(m3);
            sm.M4[k * s + j] = m4;
            sm.M4f[k * s + j] = static_cast<float>(m4);
        }
    }
    if (local == 0) {
        // C <- S C, S[i][k] = U[i][k] dv[i] (k >= i); convergence on ||C e_j||
#pragma unroll
        for (int q = 0; q < kGramRegs; ++q)
            if (threadIdx.x + q * kThreads < s * s) fs.Cl[threadIdx.x + q * kThreads] = cv[q];
        if (threadIdx.x == 0) fs.notconv = 0;
        __syncthreads();
        small_gemm<4 * NB>(
            s,
            [&](int i, int k) {
                const double v = fs.A[i * w + k] * fs.dv[i];
                return k >= i ? v : 0.0;
            },
            [&](int k, int j) { return fs.Cl[k * s + j]; }, [&](int i, int j, double v) { fs.G[i * s + j] = v; },
            [](int bi, int) { return 4 * bi; });
        __syncthreads();
        // ||C e_j|| (C upper triangular) by 8 lanes per column: rows p, p + 8,
        // p + 16, p + 24, then a fixed butterfly over the 8 lanes
        {
            static_assert(kThreads >= 8 * 32, "8 lanes per column for s <= 32");
            const int j = threadIdx.x >> 3, p = threadIdx.x & 7;
            double n = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = p + 8 * q;
                const double v = (j < s && r <= j) ? fs.G[r * s + j] : 0.0;
                n = fma(v, v, n);
            }
            n += __shfl_xor(n, 4);
            n += __shfl_xor(n, 2);
            n += __shfl_xor(n, 1);
            if (j < s && p == 0 && !(sqrt(n) <= sm.th[j])) atomicAdd(&fs.notconv, 1);
        }
        for (int e = threadIdx.x; e < s * s; e += kThreads) sm.C[e] = fs.G[e];
        __syncthreads();
        if (threadIdx.x < 64) {
            const int inactive = __popcll(__ballot(threadIdx.x < s && !fs.active[threadIdx.x]));
            if (threadIdx.x == 0) {
                ctrl[kIters] = iters + (mode == 1 ? 1 : 0);
                ctrl[kDeflated] = inactive;
                if (inactive == s) ctrl[kAllDeflated] = 1;
                if (fs.notconv == 0 || inactive == s) ctrl[kConverged] = 1;
            }
        }
    }
    __syncthreads();
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            if (tile != local || gi != 0 || wave == 0) {
                load(tile, gi);
                part_d(tile, gi);
            }
#pragma unroll
            for (int p = 0; p < PRE; ++p) {
                const int64_t r0 = tile * kTileRows + wave * 64 + (gi * PRE + p) * 16;
#pragma unroll
                for (int jb = 0; jb < NB; ++jb) {
                    const int colj = jb * 16 + li;
                    V ap;
#pragma unroll
                    for (int r = 0; r < 4; ++r) ap[r] = T(0);
                    // S^+ upper, S^T lower triangular: only their nonzero 16-row blocks
#pragma unroll
                    for (int t = 0; t < 4 * (jb + 1); ++t) ap = MF<T>::mma(wa[p][t], M3[(4 * t + lg) * MST + colj], ap);
#pragma unroll
                    for (int t = 4 * jb; t < KS; ++t) ap = MF<T>::mma(pa[p][t], M4[(4 * t + lg) * MST + colj], ap);
                    if (colj < s) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) P[colj * ldw + r0 + mfma_row<kF64>(lg, r)] = ap[r];
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ outer-loop kernels (grouped)

// R64 = B - A X in FP64 for the chip's rows (padding rows zero).
__global__ __launch_bounds__(kThreads) void residual_kernel(const ChipDev *__restrict__ cds,
                                                            const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (!cd.ctrl[kActive]) return;
    const int nx = cd.nx, ny = cd.ny, nz = cd.nz;
    const int64_t n = cd.n, ldw = cd.ldw, plane = static_cast<int64_t>(nx) * ny;
    const int64_t ntiles = ldw / kTileRows;
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        const int64_t a = tile * kTileRows + threadIdx.x;
        if (a >= n) {
            for (int c = 0; c < s; ++c) cd.R64[c * ldw + a] = 0.0;
            continue;
        }
        const int i = static_cast<int>(a % nx);
        const int64_t q = a / nx;
        const int j = static_cast<int>(q % ny);
        const int l = static_cast<int>(q / ny);
        const int64_t oxm = i > 0 ? -1 : 0, oxp = i < nx - 1 ? 1 : 0;
        const int64_t oym = j > 0 ? -static_cast<int64_t>(nx) : 0, oyp = j < ny - 1 ? nx : 0;
        const int64_t ozm = l > 0 ? -plane : 0, ozp = l < nz - 1 ? plane : 0;
        const double d = cd.d64[a];
        const double cxp = cd.x64[a], cxm = i > 0 ? cd.x64[a - 1] : 0.0;
        const double cyp = cd.y64[a], cym = j > 0 ? cd.y64[a - nx] : 0.0;
        const double czp = cd.z64[a], czm = l > 0 ? cd.z64[a - plane] : 0.0;
        for (int c = 0; c < s; ++c) {
            const double *x = cd.X + c * cd.ldx + a;
            const double nb = cxm * x[oxm] + cxp * x[oxp] + cym * x[oym] + cyp * x[oyp] + czm * x[ozm] + czp * x[ozp];
            cd.R64[c * ldw + a] = cd.B[c * cd.ldb + a] - (d * x[0] - nb);
        }
    }
}

// Per-workgroup column sums of squares of B (which = 0), R64 (which = 1) or
// S R64 (which = 2, chips under Jacobi scaling; others skip) over the chip's
// rows, into parts[local * s + c].
__global__ __launch_bounds__(kThreads) void colsq_kernel(const ChipDev *__restrict__ cds, const uint16_t *__restrict__ tab,
                                                         int s, int which)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (which >= 1 && !cd.ctrl[kActive]) return;
    if (which == 2 && !cd.scale) return;
    __shared__ double sh[kThreads / 64][kMaxS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double *src = which == 0 ? cd.B : cd.R64;
    const int64_t ld = which == 0 ? cd.ldb : cd.ldw;
    const int64_t ntiles = cd.ldw / kTileRows;
    for (int c = 0; c < s; ++c) {
        double acc = 0.0;
        for (int64_t tile = local; tile < ntiles; tile += wgs) {
            const int64_t a = tile * kTileRows + threadIdx.x;
            if (a < cd.n) {
                const double v = which == 2 ? src[c * ld + a] * cd.scale[a] : src[c * ld + a];
                acc = fma(v, v, acc);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) sh[wave][c] = acc;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < s; c += kThreads) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += sh[w][c];
        cd.parts[static_cast<size_t>(local) * s + c] = t;
    }
}

// Sum of column c over the chip's np workgroup partials (row stride ld) by
// `lanes` consecutive lanes of one wave: lane l takes partials l, l + lanes,
// ... in order, then the lanes combine in a fixed tree (deterministic).
__device__ __forceinline__ double column_partials(const double *__restrict__ parts, int np, int ld, int c, int l,
                                                  int lanes)
{
    double t = 0.0;
#pragma unroll 8
    for (int p = l; p < np; p += lanes) t += parts[static_cast<size_t>(p) * ld + c];
    for (int off = lanes / 2; off > 0; off >>= 1) t += __shfl_down(t, off, lanes);
    return t;
}

// Lanes per column for `cols` columns over one workgroup: a power of two,
// at most a wave.
__device__ __forceinline__ int lanes_per_column(int cols)
{
    int l = 64;
    while (l > 1 && l * cols > kThreads) l >>= 1;
    return l;
}

// norms[c] = sum over the chip's workgroups of the column partials (one
// workgroup per chip).
__global__ __launch_bounds__(kThreads) void colsq_reduce_kernel(const ChipDev *__restrict__ cds, int s, int which)
{
    const ChipDev &cd = cds[blockIdx.x];
    if (which >= 1 && !cd.ctrl[kActive]) return;
    if (which == 2 && !cd.scale) return;
    const int lanes = lanes_per_column(s);
    for (int c0 = 0; c0 < s; c0 += kThreads / lanes) {
        const int c = c0 + static_cast<int>(threadIdx.x) / lanes;
        const double t = column_partials(cd.parts, cd.wgs, s, c < s ? c : 0, threadIdx.x % lanes, lanes);
        if (c < s && threadIdx.x % lanes == 0) cd.norms[c] = t;
    }
}

// Inner-solve start for active chips: W = (T) R64 (S R64 under Jacobi
// scaling), D = P = AP = 0 (padding rows included); C = I and M1 = 0.
template <class T>
__global__ __launch_bounds__(kThreads) void inner_start_kernel(const ChipDev *__restrict__ cds,
                                                               const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (!cd.ctrl[kActive]) return;
    const int64_t ldw = cd.ldw, ntiles = ldw / kTileRows;
    T *W = static_cast<T *>(cd.W), *D = static_cast<T *>(cd.Dv), *P = static_cast<T *>(cd.P), *AP = static_cast<T *>(cd.AP);
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        const int64_t a = tile * kTileRows + threadIdx.x;
        const double sa = cd.scale ? (a < cd.n ? cd.scale[a] : 0.0) : 1.0;
        for (int c = 0; c < s; ++c) {
            const int64_t e = c * ldw + a;
            W[e] = static_cast<T>(cd.R64[e] * sa);
            D[e] = T(0);
            P[e] = T(0);
            AP[e] = T(0);
        }
    }
    if (local == 0) {
        for (int e = threadIdx.x; e < s * s; e += kThreads) {
            cd.sm.C[e] = (e / s == e % s) ? 1.0 : 0.0;
            cd.sm.M1[e] = 0.0;
            cd.sm.M1f[e] = 0.0f;
        }
    }
}

// X = X0 (or 0) for the chip's rows.
__global__ __launch_bounds__(kThreads) void start_x_kernel(const ChipDev *__restrict__ cds,
                                                           const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    const int64_t ntiles = cd.ldw / kTileRows;
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        const int64_t a = tile * kTileRows + threadIdx.x;
        if (a >= cd.n) continue;
        for (int c = 0; c < s; ++c) cd.X[c * cd.ldx + a] = cd.X0 ? cd.X0[c * cd.ldx0 + a] : 0.0;
    }
}

// Per-workgroup column sums of X0 . B and X0 . R64 (R64 = B - A X0) over
// the chip's rows, into parts[local * 2s + c] and parts[local * 2s + s + c].
__global__ __launch_bounds__(kThreads) void x0_dots_kernel(const ChipDev *__restrict__ cds,
                                                           const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (!cd.X0) return;
    __shared__ double sh[kThreads / 64][2 * kMaxS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t ntiles = cd.ldw / kTileRows;
    for (int c = 0; c < s; ++c) {
        double ab = 0.0, ar = 0.0;
        for (int64_t tile = local; tile < ntiles; tile += wgs) {
            const int64_t a = tile * kTileRows + threadIdx.x;
            if (a < cd.n) {
                const double x = cd.X[c * cd.ldx + a];
                ab = fma(x, cd.B[c * cd.ldb + a], ab);
                ar = fma(x, cd.R64[c * cd.ldw + a], ar);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ab += __shfl_xor(ab, off);
            ar += __shfl_xor(ar, off);
        }
        if (lane == 0) {
            sh[wave][c] = ab;
            sh[wave][s + c] = ar;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < 2 * s; c += kThreads) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += sh[w][c];
        cd.parts[static_cast<size_t>(local) * 2 * s + c] = t;
    }
}

// dots[chip * 2 kMaxS + c] = sum over the chip's workgroups, in a fixed order (one
// workgroup per chip).
__global__ __launch_bounds__(kThreads) void x0_dots_reduce_kernel(const ChipDev *__restrict__ cds, int s,
                                                                  double *__restrict__ dots)
{
    const ChipDev &cd = cds[blockIdx.x];
    if (!cd.X0) return;
    const int lanes = lanes_per_column(2 * s);
    for (int c0 = 0; c0 < 2 * s; c0 += kThreads / lanes) {
        const int c = c0 + static_cast<int>(threadIdx.x) / lanes;
        const double t = column_partials(cd.parts, cd.wgs, 2 * s, c < 2 * s ? c : 0, threadIdx.x % lanes, lanes);
        if (c < 2 * s && threadIdx.x % lanes == 0) dots[static_cast<size_t>(blockIdx.x) * 2 * kMaxS + c] = t;
    }
}

// X[:, c] *= alpha[chip * kMaxS + c] for chips that were given an initial guess.
__global__ __launch_bounds__(kThreads) void scale_cols_kernel(const ChipDev *__restrict__ cds,
                                                              const uint16_t *__restrict__ tab, int s,
                                                              const double *__restrict__ alpha)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (!cd.X0) return;
    const double *al = alpha + static_cast<size_t>(chip_index(tab)) * kMaxS;
    const int64_t ntiles = cd.ldw / kTileRows;
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        const int64_t a = tile * kTileRows + threadIdx.x;
        if (a >= cd.n) continue;
        for (int c = 0; c < s; ++c) cd.X[c * cd.ldx + a] *= al[c];
    }
}

// X (FP64) += D (type T), or S D under Jacobi scaling, for active chips.
template <class T>
__global__ __launch_bounds__(kThreads) void add_out_kernel(const ChipDev *__restrict__ cds,
                                                           const uint16_t *__restrict__ tab, int s)
{
    int local;
    const ChipDev &cd = chip_of(cds, tab, local);
    const int wgs = cd.wgs;
    if (!cd.ctrl[kActive]) return;
    const T *D = static_cast<const T *>(cd.Dv);
    const int64_t ntiles = cd.ldw / kTileRows;
    for (int64_t tile = local; tile < ntiles; tile += wgs) {
        const int64_t a = tile * kTileRows + threadIdx.x;
        if (a >= cd.n) continue;
        const double sa = cd.scale ? cd.scale[a] : 1.0;
        for (int c = 0; c < s; ++c) cd.X[c * cd.ldx + a] += sa * static_cast<double>(D[c * cd.ldw + a]);
    }
}

// prog[chip] = max_j ||C e_j|| / th_j, the inner solve's residual over its
// target (||r_j|| = ||C e_j||), or 0 for a chip that has converged (one
// wavefront per chip).
__global__ __launch_bounds__(64) void progress_kernel(const ChipDev *__restrict__ cds, int s, double *__restrict__ prog)
{
    const ChipDev &cd = cds[blockIdx.x];
    const int lane = threadIdx.x;
    double q = 0.0;
    if (!cd.ctrl[kConverged] && lane < s) {
        double n2 = 0.0;
        for (int r = 0; r < s; ++r) n2 = fma(cd.sm.C[r * s + lane], cd.sm.C[r * s + lane], n2);
        q = sqrt(n2) / cd.sm.th[lane];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q = fmax(q, __shfl_xor(q, off));
    if (lane == 0) prog[blockIdx.x] = cd.ctrl[kConverged] ? 0.0 : q;
}

// ------------------------------------------------------------------ host side

inline int nb_for(int s) { return (s + 15) / 16; }

// Workspace layout of a batch: a header (chip table, workgroup table,
// thresholds, control words, norms) and one region per chip.
struct ChipHost {
    const Operator *op;
    int64_t n, ldw;
    int tiles, wgs, wg_base;
    size_t off;  // chip region
};

struct Layout {
    int nchips = 0, s = 0, total_wgs = 0, tiles_per_wg = 1;
    int nx_align = 4;  // largest of 1, 2, 4 dividing every chip's nx
    bko_dtype compute = BKO_F64;
    size_t off_cds = 0, off_tab = 0, off_th = 0, off_ctrl = 0, off_norms = 0, off_alpha = 0, off_dots = 0, off_prog = 0,
           bytes = 0;
    std::vector<ChipHost> chips;
};

// Gram partials a chip may produce per reduction: enough for one workgroup
// per row tile of the chips in use, bounded so a chip's partials stay within
// 32 MB at any s.
inline int part_cap(int s) { return std::max(512, (1 << 22) / (s * s)); }
inline int max_parts(int tiles, int s) { return std::min(tiles, part_cap(s)); }

inline size_t chip_region_bytes(int64_t ldw, int s, bko_dtype compute, size_t *offs)
{
    const size_t nparts = static_cast<size_t>(max_parts(static_cast<int>(ldw / kTileRows), s));
    const size_t vsz = compute == BKO_F64 ? 8 : 4;
    const size_t ss = static_cast<size_t>(s) * s;
    const size_t sizes[] = {sizeof(double) * ldw * s,                     // R64
                            vsz * ldw * s, vsz * ldw * s, vsz * ldw * s,  // Dv, P, AP
                            vsz * ldw * s,                                // W
                            sizeof(double) * ss * 5,                      // C, M1..M4
                            sizeof(double) * kMaxS,                       // (unused slot)
                            sizeof(float) * ss * 4,                       // M1f..M4f
                            sizeof(double) * std::max<size_t>(ss, 2 * s) * nparts,  // parts (Gram, or 2 column sums)
                            sizeof(double) * ss};                         // gram
    size_t o = 0;
    for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
        if (offs) offs[k] = o;
        o = align_up(o + sizes[k], 256);
    }
    return o;
}

// tiles_per_wg: row tiles each workgroup of the row kernels walks (the
// autotuned granularity); a chip gets ceil(tiles / tiles_per_wg) workgroups,
// at most max_parts of them.
Layout make_layout(const Operator *const *ops, int nchips, int s, bko_dtype compute, int tiles_per_wg)
{
    Layout L;
    L.nchips = nchips;
    L.s = s;
    L.compute = compute;
    L.tiles_per_wg = tiles_per_wg;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t q = o;
        o = align_up(o + bytes, 256);
        return q;
    };
    L.off_cds = take(sizeof(ChipDev) * nchips);
    int total = 0;
    L.chips.resize(nchips);
    for (int c = 0; c < nchips; ++c) {
        ChipHost &h = L.chips[c];
        h.op = ops[c];
        h.n = ops[c]->n;
        h.ldw = static_cast<int64_t>(align_up(static_cast<size_t>(h.n), kTileRows));
        h.tiles = static_cast<int>(h.ldw / kTileRows);
        h.wgs = std::min((h.tiles + tiles_per_wg - 1) / tiles_per_wg, max_parts(h.tiles, s));
        h.wg_base = total;
        total += h.wgs;
        while (ops[c]->nx % L.nx_align != 0) L.nx_align /= 2;
    }
    L.total_wgs = total;
    int table = 0;  // sized for one tile per workgroup, so offsets do not depend on the tuning
    for (int c = 0; c < nchips; ++c) table += max_parts(L.chips[c].tiles, s);
    L.off_tab = take(sizeof(uint16_t) * table);
    L.off_th = take(sizeof(double) * kMaxS * nchips);
    L.off_ctrl = take(sizeof(int) * kCtrlInts * nchips);
    L.off_norms = take(sizeof(double) * kMaxS * nchips);
    L.off_alpha = take(sizeof(double) * kMaxS * nchips);
    L.off_dots = take(sizeof(double) * 2 * kMaxS * nchips);
    L.off_prog = take(sizeof(double) * nchips);
    for (int c = 0; c < nchips; ++c) L.chips[c].off = take(chip_region_bytes(L.chips[c].ldw, s, compute, nullptr));
    L.bytes = o;
    return L;
}

// Device chip records for one call.
std::vector<ChipDev> chip_records(const Layout &L, void *work, const double *const *B, const int64_t *ldb,
                                  double *const *X, const int64_t *ldx, const double *const *X0, const int64_t *ldx0)
{
    char *base = static_cast<char *>(work);
    const bool f64 = L.compute == BKO_F64;
    const size_t ss = static_cast<size_t>(L.s) * L.s;
    std::vector<ChipDev> v(L.nchips);
    for (int c = 0; c < L.nchips; ++c) {
        const ChipHost &h = L.chips[c];
        const Operator &op = *h.op;
        ChipDev &d = v[c];
        std::memset(&d, 0, sizeof(d));
        if (op.precond == BKO_PRECOND_JACOBI) {
            d.cdiag = f64 ? static_cast<const void *>(op.sdiag64) : static_cast<const void *>(op.sdiag32);
            d.cwx = f64 ? static_cast<const void *>(op.swx64) : static_cast<const void *>(op.swx32);
            d.cwy = f64 ? static_cast<const void *>(op.swy64) : static_cast<const void *>(op.swy32);
            d.cwz = f64 ? static_cast<const void *>(op.swz64) : static_cast<const void *>(op.swz32);
            d.scale = op.scale64;
        } else {
            d.cdiag = f64 ? static_cast<const void *>(op.diag64) : static_cast<const void *>(op.diag32);
            d.cwx = f64 ? static_cast<const void *>(op.wx64) : static_cast<const void *>(op.wx32);
            d.cwy = f64 ? static_cast<const void *>(op.wy64) : static_cast<const void *>(op.wy32);
            d.cwz = f64 ? static_cast<const void *>(op.wz64) : static_cast<const void *>(op.wz32);
            d.scale = nullptr;
        }
        d.d64 = op.diag64;
        d.x64 = op.wx64;
        d.y64 = op.wy64;
        d.z64 = op.wz64;
        d.nx = op.nx;
        d.ny = op.ny;
        d.nz = op.nz;
        d.wgs = h.wgs;
        d.n = h.n;
        d.ldw = h.ldw;
        d.wg_base = h.wg_base;
        d.B = B ? B[c] : nullptr;
        d.ldb = ldb ? ldb[c] : 0;
        d.X = X ? X[c] : nullptr;
        d.ldx = ldx ? ldx[c] : 0;
        d.X0 = X0 ? X0[c] : nullptr;
        d.ldx0 = ldx0 ? ldx0[c] : 0;
        size_t off[10];
        chip_region_bytes(h.ldw, L.s, L.compute, off);
        char *r = base + h.off;
        d.R64 = reinterpret_cast<double *>(r + off[0]);
        d.Dv = r + off[1];
        d.P = r + off[2];
        d.AP = r + off[3];
        d.W = r + off[4];
        double *sm = reinterpret_cast<double *>(r + off[5]);
        d.sm.C = sm;
        d.sm.M1 = sm + ss;
        d.sm.M2 = sm + 2 * ss;
        d.sm.M3 = sm + 3 * ss;
        d.sm.M4 = sm + 4 * ss;
        float *smf = reinterpret_cast<float *>(r + off[7]);
        d.sm.M1f = smf;
        d.sm.M2f = smf + ss;
        d.sm.M3f = smf + 2 * ss;
        d.sm.M4f = smf + 3 * ss;
        d.sm.th = reinterpret_cast<double *>(base + L.off_th) + static_cast<size_t>(c) * kMaxS;
        d.parts = reinterpret_cast<double *>(r + off[8]);
        d.gram = reinterpret_cast<double *>(r + off[9]);
        d.norms = reinterpret_cast<double *>(base + L.off_norms) + static_cast<size_t>(c) * kMaxS;
        d.ctrl = reinterpret_cast<int *>(base + L.off_ctrl) + static_cast<size_t>(c) * kCtrlInts;
    }
    return v;
}

std::vector<uint16_t> wg_table(const Layout &L)
{
    std::vector<uint16_t> t(L.total_wgs);
    for (int c = 0; c < L.nchips; ++c)
        for (int g = 0; g < L.chips[c].wgs; ++g) t[L.chips[c].wg_base + g] = static_cast<uint16_t>(c);
    return t;
}

// Kernel launch context of one batch call.
struct Ctx {
    const Layout *L;
    const ChipDev *cds;
    const uint16_t *tab;
    hipStream_t st;
};

template <class T, int NB>
bko_status launch_row_kernels(int which, const Ctx &x, int init)
{
    const int s = x.L->s;
    const dim3 grid(static_cast<unsigned>(x.L->total_wgs)), block(kThreads);
    if (which == 0) {
        TimedLaunch tl(kSpmm, x.st);
        if (x.L->nx_align % vec_cells<T>() == 0)
            tl.launch(spmm_gram_vec_kernel<T, NB>, grid, dim3(kSpThreads), spmm_gram_lds<T, NB>(), x.cds, x.tab, s);
        else
            tl.launch(spmm_gram_kernel<T, NB>, grid, dim3(kSpThreads), spmm_gram_lds<T, NB>(), x.cds, x.tab, s);
    } else if (which == 1) {
        TimedLaunch tl(kUpdate, x.st);
        if constexpr (sizeof(T) == 4 && NB > 2)
            tl.launch(update_w_rows2_kernel<NB>, grid, block, 0, x.cds, x.tab, s, init);
        else
            tl.launch(update_w_kernel<T, NB>, grid, block, 0, x.cds, x.tab, s, init);
    } else {
        TimedLaunch tl(::bko::kUpdateDQP, x.st);
        const size_t sp = 16 * NB;
        if constexpr (sizeof(T) == 4 && NB > 2)
            tl.launch(update_dqp_rows4_kernel<NB>, grid, block, static_cast<uint32_t>(3 * sizeof(T) * sp * (sp + 1)),
                      x.cds, x.tab, s);
        else
            tl.launch(update_dqp_kernel<T, NB>, grid, block, static_cast<uint32_t>(3 * sizeof(T) * sp * (sp + 1)),
                      x.cds, x.tab, s);
    }
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class T>
bko_status launch_row(int which, const Ctx &x, int init)
{
    switch (nb_for(x.L->s)) {
    case 1: return launch_row_kernels<T, 1>(which, x, init);
    case 2: return launch_row_kernels<T, 2>(which, x, init);
    case 3: return launch_row_kernels<T, 3>(which, x, init);
    default: return launch_row_kernels<T, 4>(which, x, init);
    }
}

// Largest LDS request of the row kernels at this s and precision.
size_t row_kernel_lds(int s, bko_dtype compute)
{
    const int nb = nb_for(s);
    const size_t sp = 16 * nb;
    const size_t vsz = compute == BKO_F64 ? 8 : 4;
    size_t g;
    if (compute == BKO_F64) g = nb == 1 ? spmm_gram_lds<double, 1>() : nb == 2 ? spmm_gram_lds<double, 2>()
                                : nb == 3 ? spmm_gram_lds<double, 3>() : spmm_gram_lds<double, 4>();
    else g = nb == 1 ? spmm_gram_lds<float, 1>() : nb == 2 ? spmm_gram_lds<float, 2>()
             : nb == 3 ? spmm_gram_lds<float, 3>() : spmm_gram_lds<float, 4>();
    const size_t w = 2 * vsz * sp * (sp + 1) + sizeof(double) * kMaxS * kMaxS;
    const size_t dqp = 3 * vsz * sp * (sp + 1);
    return std::max(g, std::max(w, dqp));
}

// reduce the partials of the last Gram step of every chip, then factor
bko_status launch_reduce_factor(const Ctx &x, double rel_thr, int mode)
{
    const int s = x.L->s, ss = s * s;
    BKO_CHECK(s > 32 && s <= kMaxS, "the separate factorisation kernel is for 32 < s <= 64, got s = %d", s);
    TimedLaunch tl(kSmall, x.st);
    const unsigned rblocks = static_cast<unsigned>(std::min(kRedBlocks, ss));
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(rblocks, static_cast<unsigned>(x.L->nchips)), dim3(kThreads), 0, x.st,
                       x.cds, ss);
    BKO_HIP(hipGetLastError());
    const size_t lds = sizeof(double) * 4 * ss;  // [U | E], the Gram, C
    const dim3 grid(static_cast<unsigned>(x.L->nchips));
    hipLaunchKernelGGL(factor_kernel, grid, dim3(kFacThreads), lds, x.st, x.cds, s, rel_thr, mode);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

// s <= 32: the factorisations run inside the update kernels
inline bool fused_factor(int s) { return s <= 32; }

bko_status launch_reduce(const Ctx &x)
{
    const int ss = x.L->s * x.L->s;
    TimedLaunch tl(kSmall, x.st);
    const unsigned rblocks = static_cast<unsigned>(std::min(kRedBlocks, ss));
    tl.launch(gram_reduce_kernel, dim3(rblocks, static_cast<unsigned>(x.L->nchips)), dim3(kThreads), 0, x.cds, ss);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

// which 1: W update with delta^+ factored in; 2: D, P update with the QR of
// W factored in (mode 1, or 2 for an inner solve's first QR)
template <class T, int NB>
bko_status launch_fused_kernel(int which, const Ctx &x, double rel_thr, int mode)
{
    const dim3 grid(static_cast<unsigned>(x.L->total_wgs)), block(kThreads);
    const int s = x.L->s;
    if (which == 1) {
        TimedLaunch tl(kUpdate, x.st);
        tl.launch(update_w_fused_kernel<T, NB>, grid, block, 0, x.cds, x.tab, s, rel_thr);
    } else {
        TimedLaunch tl(::bko::kUpdateDQP, x.st);
        tl.launch(update_dqp_fused_kernel<T, NB>, grid, block, 0, x.cds, x.tab, s, rel_thr, mode);
    }
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class T>
bko_status launch_fused(int which, const Ctx &x, double rel_thr, int mode)
{
    return nb_for(x.L->s) == 1 ? launch_fused_kernel<T, 1>(which, x, rel_thr, mode)
                               : launch_fused_kernel<T, 2>(which, x, rel_thr, mode);
}

// One block iteration for every chip of the batch.
template <class T>
bko_status iteration(const Ctx &x, double rel_thr)
{
    bko_status rc;
    if ((rc = launch_row<T>(0, x, 0)) != BKO_OK) return rc;
    if (fused_factor(x.L->s)) {
        if ((rc = launch_reduce(x)) != BKO_OK) return rc;
        if ((rc = launch_fused<T>(1, x, rel_thr, 0)) != BKO_OK) return rc;
        if ((rc = launch_reduce(x)) != BKO_OK) return rc;
        return launch_fused<T>(2, x, rel_thr, 1);
    }
    if ((rc = launch_reduce_factor(x, rel_thr, 0)) != BKO_OK) return rc;
    if ((rc = launch_row<T>(1, x, 0)) != BKO_OK) return rc;
    if ((rc = launch_reduce_factor(x, rel_thr, 1)) != BKO_OK) return rc;
    return launch_row<T>(2, x, 0);
}

template <class T>
bko_status run_chunk(const Ctx &x, double rel_thr, int len, GraphCache *gc, void *work)
{
    const bool graph = gc != nullptr && x.st != nullptr && !timing_active();
    if (!graph) {
        for (int it = 0; it < len; ++it) {
            bko_status rc = iteration<T>(x, rel_thr);
            if (rc != BKO_OK) return rc;
        }
        return BKO_OK;
    }
    if (gc->work != work) gc->clear();
    gc->work = work;
    // a chunk of any length replays the graphs of its binary digits, so at
    // most seven graphs (1, 2, 4, ..., 64 iterations) are ever captured
    for (int bit = 64; bit >= 1; bit >>= 1) {
        if (!(len & bit)) continue;
        auto found = gc->execs.find(bit);
        if (found == gc->execs.end()) {
            BKO_HIP(hipStreamBeginCapture(x.st, hipStreamCaptureModeThreadLocal));
            bko_status rc = BKO_OK;
            for (int it = 0; it < bit && rc == BKO_OK; ++it) rc = iteration<T>(x, rel_thr);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(x.st, &g);
            if (rc != BKO_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            hipGraphExec_t ex = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
            found = gc->execs.emplace(bit, ex).first;
        }
        BKO_HIP(hipGraphLaunch(found->second, x.st));
    }
    return BKO_OK;
}

struct ChipState {
    bko_solve_info info{};
    double prev_rel = HUGE_VAL;
    int stagnant = 0;
    bool done = false;
    std::vector<double> bnorm, rnorm;
};

// Squared column norms of B (which = 0) or of the active chips' residuals
// (which = 1) into each chip's norms slot.
bko_status host_norms(const Ctx &x, int which)
{
    const Layout &L = *x.L;
    hipLaunchKernelGGL(colsq_kernel, dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, x.st, x.cds, x.tab, L.s,
                       which);
    BKO_HIP(hipGetLastError());
    hipLaunchKernelGGL(colsq_reduce_kernel, dim3(static_cast<unsigned>(L.nchips)), dim3(kThreads), 0, x.st, x.cds, L.s,
                       which);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class T>
bko_status batch_solve_t(const Layout &L, void *work, const double *const *B, const int64_t *ldb, double *const *X,
                         const int64_t *ldx, const double *const *X0, const int64_t *ldx0, double tol, int max_iter,
                         bko_solve_info *infos, hipStream_t st, GraphCache *gc)
{
    const int s = L.s, nc = L.nchips;
    char *base = static_cast<char *>(work);
    const bool f64 = sizeof(T) == 8;
    const double rel_thr = f64 ? 1e-13 : 1e-12;
    const double inner_rel_f32 = 1e-5;
    if (row_kernel_lds(s, L.compute) > device_max_lds()) {
        set_error("s = %d needs %zu bytes of LDS per workgroup in this precision; the device grants %zu", s,
                  row_kernel_lds(s, L.compute), device_max_lds());
        return BKO_EINVAL;
    }
    // chip records and the workgroup table (host copies live until the final synchronisation)
    const std::vector<ChipDev> recs = chip_records(L, work, B, ldb, X, ldx, X0, ldx0);
    bool any_scaled = false;
    for (const ChipDev &r : recs) any_scaled = any_scaled || r.scale != nullptr;
    const std::vector<uint16_t> tabh = wg_table(L);
    std::vector<int> ctrlh(static_cast<size_t>(kCtrlInts) * nc, 0);
    std::vector<double> thh(static_cast<size_t>(kMaxS) * nc, 0.0), nh(static_cast<size_t>(kMaxS) * nc, 0.0),
        sh(static_cast<size_t>(kMaxS) * nc, 0.0);
    Ctx x{&L, reinterpret_cast<const ChipDev *>(base + L.off_cds),
          L.nchips == 1 ? nullptr : reinterpret_cast<const uint16_t *>(base + L.off_tab), st};
    int *ctrl_d = reinterpret_cast<int *>(base + L.off_ctrl);
    double *th_d = reinterpret_cast<double *>(base + L.off_th);
    double *norms_d = reinterpret_cast<double *>(base + L.off_norms);
    BKO_HIP(hipMemcpyAsync(base + L.off_cds, recs.data(), sizeof(ChipDev) * nc, hipMemcpyHostToDevice, st));
    BKO_HIP(hipMemcpyAsync(base + L.off_tab, tabh.data(), sizeof(uint16_t) * tabh.size(), hipMemcpyHostToDevice, st));
    // every chip active for the start: ||b_j||, X = X0 or 0
    for (int c = 0; c < nc; ++c) ctrlh[static_cast<size_t>(c) * kCtrlInts + kActive] = 1;
    BKO_HIP(hipMemcpyAsync(ctrl_d, ctrlh.data(), sizeof(int) * ctrlh.size(), hipMemcpyHostToDevice, st));
    bko_status rc;
    if ((rc = host_norms(x, 0)) != BKO_OK) return rc;
    std::vector<double> bn(static_cast<size_t>(kMaxS) * nc);
    BKO_HIP(hipMemcpyAsync(bn.data(), norms_d, sizeof(double) * bn.size(), hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(start_x_kernel, dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, st, x.cds, x.tab, s);
    BKO_HIP(hipGetLastError());
    BKO_HIP(hipStreamSynchronize(st));
    std::vector<ChipState> cs(nc);
    for (int c = 0; c < nc; ++c) {
        cs[c].info.status = BKO_ENOCONV;
        cs[c].bnorm.resize(s);
        for (int j = 0; j < s; ++j) cs[c].bnorm[j] = std::sqrt(bn[static_cast<size_t>(c) * kMaxS + j]);
        for (int j = 0; j < s; ++j)
            if (!std::isfinite(cs[c].bnorm[j])) {
                set_error("right-hand side column %d of chip %d is not finite", j, c);
                return BKO_EINVAL;
            }
    }
    // an initial guess column x0 is replaced by alpha x0 with alpha =
    // x0'b / x0'A x0, the multiple of x0 closest to the solution in the A-norm
    // (the norm block CG minimises), which is never further than the zero
    // start; a column with alpha <= 0 or not finite starts from zero
    bool any_x0 = false;
    for (int c = 0; c < nc; ++c) any_x0 = any_x0 || recs[c].X0 != nullptr;
    if (any_x0) {
        hipLaunchKernelGGL(residual_kernel, dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, st, x.cds, x.tab,
                           s);
        BKO_HIP(hipGetLastError());
        double *dots_d = reinterpret_cast<double *>(base + L.off_dots);
        hipLaunchKernelGGL(x0_dots_kernel, dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, st, x.cds, x.tab,
                           s);
        BKO_HIP(hipGetLastError());
        hipLaunchKernelGGL(x0_dots_reduce_kernel, dim3(static_cast<unsigned>(nc)), dim3(kThreads), 0, st, x.cds, s, dots_d);
        BKO_HIP(hipGetLastError());
        std::vector<double> dh(static_cast<size_t>(2 * kMaxS) * nc, 0.0), alpha(static_cast<size_t>(kMaxS) * nc, 1.0);
        BKO_HIP(hipMemcpyAsync(dh.data(), dots_d, sizeof(double) * dh.size(), hipMemcpyDeviceToHost, st));
        BKO_HIP(hipStreamSynchronize(st));
        for (int c = 0; c < nc; ++c) {
            if (!recs[c].X0) continue;
            for (int j = 0; j < s; ++j) {
                const double xb = dh[static_cast<size_t>(c) * 2 * kMaxS + j];
                const double xr = dh[static_cast<size_t>(c) * 2 * kMaxS + s + j];
                const double xax = xb - xr;  // x0' A x0 = x0' (b - r0)
                double a = (xb > 0.0 && xax > 0.0) ? xb / xax : 0.0;
                if (!std::isfinite(a)) a = 0.0;
                alpha[static_cast<size_t>(c) * kMaxS + j] = a;
                if (a == 0.0) cs[c].info.x0_rejected += 1;
            }
        }
        BKO_HIP(hipMemcpyAsync(base + L.off_alpha, alpha.data(), sizeof(double) * alpha.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(scale_cols_kernel, dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, st, x.cds,
                           x.tab, s, reinterpret_cast<const double *>(base + L.off_alpha));
        BKO_HIP(hipGetLastError());
        BKO_HIP(hipStreamSynchronize(st));
    }

    for (int outer = 0; outer < 100; ++outer) {
        // R = B - A X in FP64 and its column norms, for the chips still running
        {
            TimedLaunch tl(kResid, st);
            tl.launch(residual_kernel, dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, x.cds, x.tab, s);
            BKO_HIP(hipGetLastError());
        }
        if ((rc = host_norms(x, 1)) != BKO_OK) return rc;
        BKO_HIP(hipMemcpyAsync(nh.data(), norms_d, sizeof(double) * nh.size(), hipMemcpyDeviceToHost, st));
        if (any_scaled) {
            // norms of S R for the chips under Jacobi scaling (their inner
            // solves measure the scaled residual)
            if ((rc = host_norms(x, 2)) != BKO_OK) return rc;
            BKO_HIP(hipMemcpyAsync(sh.data(), norms_d, sizeof(double) * sh.size(), hipMemcpyDeviceToHost, st));
        }
        BKO_HIP(hipStreamSynchronize(st));
        int active = 0;
        for (int c = 0; c < nc; ++c) {
            ChipState &k = cs[c];
            int *ch = &ctrlh[static_cast<size_t>(c) * kCtrlInts];
            std::fill(ch, ch + kCtrlInts, 0);
            if (k.done) {
                ch[kConverged] = ch[kStop] = 1;
                continue;
            }
            k.rnorm.resize(s);
            double rel = 0.0;
            bool finite = true;
            for (int j = 0; j < s; ++j) {
                k.rnorm[j] = std::sqrt(nh[static_cast<size_t>(c) * kMaxS + j]);
                finite = finite && std::isfinite(k.rnorm[j]);
                const double bj = k.bnorm[j];
                rel = std::max(rel, bj > 0 ? k.rnorm[j] / bj : (k.rnorm[j] > 0 ? HUGE_VAL : 0.0));
            }
            k.info.max_rel_res = rel;
            int status = -1;
            if (!finite) status = BKO_EINVAL;
            else if (rel <= tol) status = BKO_OK;
            else if (k.info.iters >= max_iter) status = BKO_ENOCONV;
            else if (rel > 0.5 * k.prev_rel && ++k.stagnant >= 3) status = BKO_EBREAKDOWN;
            if (status < 0 && rel <= 0.5 * k.prev_rel) k.stagnant = 0;
            if (status >= 0) {
                k.info.status = status;
                k.done = true;
                ch[kConverged] = ch[kStop] = 1;
                continue;
            }
            k.prev_rel = rel;
            ch[kActive] = 1;
            ++active;
            for (int j = 0; j < s; ++j) {
                // under Jacobi scaling the inner target is the scaled one,
                // by the ratio of the scaled to the unscaled residual norm at
                // the start (the FP64 loop checks the unscaled residual)
                double rn = k.rnorm[j], ratio = 1.0;
                if (recs[c].scale) {
                    rn = std::sqrt(sh[static_cast<size_t>(c) * kMaxS + j]);
                    ratio = k.rnorm[j] > 0.0 ? rn / k.rnorm[j] : 1.0;
                }
                const double target = 0.5 * tol * k.bnorm[j] * ratio;
                thh[static_cast<size_t>(c) * kMaxS + j] = f64 ? target : std::max(target, inner_rel_f32 * rn);
            }
        }
        if (active == 0) break;
        BKO_HIP(hipMemcpyAsync(th_d, thh.data(), sizeof(double) * thh.size(), hipMemcpyHostToDevice, st));
        BKO_HIP(hipMemcpyAsync(ctrl_d, ctrlh.data(), sizeof(int) * ctrlh.size(), hipMemcpyHostToDevice, st));
        // inner solve on A D = R: W = R, first QR, Q = W S^+, P = Q, D = 0
        hipLaunchKernelGGL((inner_start_kernel<T>), dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, st, x.cds,
                           x.tab, s);
        BKO_HIP(hipGetLastError());
        if ((rc = launch_row<T>(1, x, 1)) != BKO_OK) return rc;
        if (fused_factor(s)) {
            if ((rc = launch_reduce(x)) != BKO_OK) return rc;
            if ((rc = launch_fused<T>(2, x, rel_thr, 2)) != BKO_OK) return rc;
        } else {
            if ((rc = launch_reduce_factor(x, rel_thr, 2)) != BKO_OK) return rc;
            if ((rc = launch_row<T>(2, x, 0)) != BKO_OK) return rc;
        }
        int budget = 0;
        for (int c = 0; c < nc; ++c)
            if (!cs[c].done) budget = std::max(budget, max_iter - cs[c].info.iters);
        // chunk lengths between convergence checks: each check also reads
        // every chip's residual-over-target ratio; from its decay over the
        // last chunk the next chunk runs the predicted remaining iterations
        // (at most 64), so few launches past convergence are wasted
        int launched = 0, chunk = 4;
        std::vector<int> hc(ctrlh.size());
        std::vector<double> prog(static_cast<size_t>(nc), 0.0), prev(static_cast<size_t>(nc), 0.0);
        for (int c = 0; c < nc; ++c) {
            if (cs[c].done) continue;
            double q = 0.0;
            for (int j = 0; j < s; ++j) {
                const double t = thh[static_cast<size_t>(c) * kMaxS + j];
                const double rn = recs[c].scale ? std::sqrt(sh[static_cast<size_t>(c) * kMaxS + j]) : cs[c].rnorm[j];
                if (t > 0.0) q = std::max(q, rn / t);
            }
            prev[c] = q;
        }
        double *prog_d = reinterpret_cast<double *>(base + L.off_prog);
        while (true) {
            const int todo = std::min(chunk, budget - launched);
            if ((rc = run_chunk<T>(x, rel_thr, todo, gc, work)) != BKO_OK) return rc;
            launched += todo;
            hipLaunchKernelGGL(progress_kernel, dim3(static_cast<unsigned>(nc)), dim3(64), 0, st, x.cds, s, prog_d);
            BKO_HIP(hipGetLastError());
            BKO_HIP(hipMemcpyAsync(hc.data(), ctrl_d, sizeof(int) * hc.size(), hipMemcpyDeviceToHost, st));
            BKO_HIP(hipMemcpyAsync(prog.data(), prog_d, sizeof(double) * prog.size(), hipMemcpyDeviceToHost, st));
            BKO_HIP(hipStreamSynchronize(st));
            int predicted = 0;
            bool known = true;
            for (int c = 0; c < nc; ++c) {
                if (cs[c].done || hc[static_cast<size_t>(c) * kCtrlInts + kConverged]) continue;
                const double q = prog[c], q0 = prev[c];
                prev[c] = q;
                if (!(q > 1.0) || !(q0 > q) || !std::isfinite(q0)) {
                    known = known && q > 0.0 && q <= 1.0;
                    continue;
                }
                const double rate = std::log(q0 / q) / todo;  // per iteration
                const double more = std::ceil(std::log(q) / rate) + 1.0;
                predicted = std::max(predicted, static_cast<int>(std::min(more, 64.0)));
            }
            const int next = known && predicted > 0 ? predicted : std::min(chunk * 2, 64);
            bool all = true, capped = false;
            for (int c = 0; c < nc; ++c) {
                if (cs[c].done) continue;
                const int *h = &hc[static_cast<size_t>(c) * kCtrlInts];
                if (!h[kConverged]) {
                    all = false;
                    // a chip at its own iteration limit is stopped here
                    if (cs[c].info.iters + h[kIters] >= max_iter) {
                        const int stop[2] = {1, 1};
                        BKO_HIP(hipMemcpyAsync(ctrl_d + static_cast<size_t>(c) * kCtrlInts + kConverged, stop,
                                               sizeof(stop), hipMemcpyHostToDevice, st));
                        capped = true;
                    }
                }
            }
            if (capped) BKO_HIP(hipStreamSynchronize(st));
            if (all || launched >= budget) break;
            chunk = std::max(1, next);
        }
        for (int c = 0; c < nc; ++c) {
            if (cs[c].done) continue;
            const int *h = &hc[static_cast<size_t>(c) * kCtrlInts];
            cs[c].info.iters += h[kIters];
            cs[c].info.refinements += 1;
            cs[c].info.deflated = std::max(cs[c].info.deflated, h[kDeflated]);
        }
        hipLaunchKernelGGL((add_out_kernel<T>), dim3(static_cast<unsigned>(L.total_wgs)), dim3(kThreads), 0, st, x.cds,
                           x.tab, s);
        BKO_HIP(hipGetLastError());
    }
    BKO_HIP(hipStreamSynchronize(st));
    bko_status worst = BKO_OK;
    for (int c = 0; c < nc; ++c) {
        if (!cs[c].done) cs[c].info.status = BKO_ENOCONV;
        if (infos) infos[c] = cs[c].info;
        if (cs[c].info.status != BKO_OK && worst == BKO_OK) worst = static_cast<bko_status>(cs[c].info.status);
    }
    if (worst == BKO_ENOCONV) set_error("no convergence within %d iterations", max_iter);
    if (worst == BKO_EBREAKDOWN) set_error("block iteration stagnated");
    if (worst == BKO_EINVAL) set_error("residual is not finite (initial guess or operator invalid)");
    return worst;
}

}  // namespace

// ------------------------------------------------------------------ public entry points

size_t solve_workspace_bytes(int64_t n, int s, bko_dtype compute)
{
    Operator op{};
    op.n = n;
    const Operator *ops[1] = {&op};
    return make_layout(ops, 1, s, compute, 1).bytes;
}

// Row tiles per workgroup of a single-chip solve: about two workgroups per
// compute unit, the granularity the batch autotuner picks on the stacks
// measured (512 tiles: one per workgroup; 4096 tiles at s = 64: eight, a
// 587 ms solve against 616 ms at one per workgroup).  The workspace is sized
// for one tile per workgroup, so any granularity fits it.
int solve_tiles_per_wg(const Operator &op)
{
    const int64_t tiles = static_cast<int64_t>(align_up(static_cast<size_t>(op.n), kTileRows)) / kTileRows;
    const int64_t target = 2 * static_cast<int64_t>(device_cu_count());
    return static_cast<int>(std::max<int64_t>(1, (tiles + target - 1) / target));
}

bko_status block_solve(const Operator &op, int s, const double *B, int64_t ldb, double *X, int64_t ldx,
                       const double *X0, int64_t ldx0, bko_dtype compute, double tol, int max_iter, void *work,
                       size_t work_bytes, bko_solve_info *info, hipStream_t st)
{
    (void)work_bytes;
    const Operator *ops[1] = {&op};
    const Layout L = make_layout(ops, 1, s, compute, solve_tiles_per_wg(op));
    const double *Bs[1] = {B};
    double *Xs[1] = {X};
    const double *X0s[1] = {X0};
    const int64_t lb[1] = {ldb}, lx[1] = {ldx}, lx0[1] = {ldx0};
    if (compute == BKO_F64)
        return batch_solve_t<double>(L, work, Bs, lb, Xs, lx, X0s, lx0, tol, max_iter, info, st, nullptr);
    return batch_solve_t<float>(L, work, Bs, lb, Xs, lx, X0s, lx0, tol, max_iter, info, st, nullptr);
}

size_t batch_solve_bytes(const BatchPlan &p)
{
    return make_layout(p.ops.data(), static_cast<int>(p.ops.size()), p.s, p.compute, 1).bytes;
}

size_t batch_workspace_bytes(const BatchPlan &p)
{
    size_t b = batch_solve_bytes(p);
    if (!p.m.empty()) {
        const int nc = static_cast<int>(p.ops.size());
        b = align_up(b + stencil_group_job_bytes(nc), 256);
        b = align_up(b + combine_group_job_bytes(nc), 256);
    }
    return b;
}

namespace {

// Time the partial-producing row kernels (stencil + Gram, and the W^T W
// Gram) at one granularity: a pass over the whole batch, plus a pass in
// which only the largest chip runs (the tail of a batch solve, where the
// slowest chips iterate alone).  Milliseconds per pass, summed.
template <class T>
bko_status time_granularity(const BatchPlan &p, int tpw, void *work, hipStream_t st, float &ms)
{
    const int nc = static_cast<int>(p.ops.size());
    const Layout L = make_layout(p.ops.data(), nc, p.s, p.compute, tpw);
    char *base = static_cast<char *>(work);
    const std::vector<ChipDev> recs = chip_records(L, work, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    const std::vector<uint16_t> tabh = wg_table(L);
    BKO_HIP(hipMemcpyAsync(base + L.off_cds, recs.data(), sizeof(ChipDev) * nc, hipMemcpyHostToDevice, st));
    BKO_HIP(hipMemcpyAsync(base + L.off_tab, tabh.data(), sizeof(uint16_t) * tabh.size(), hipMemcpyHostToDevice, st));
    Ctx x{&L, reinterpret_cast<const ChipDev *>(base + L.off_cds),
          L.nchips == 1 ? nullptr : reinterpret_cast<const uint16_t *>(base + L.off_tab), st};
    int biggest = 0;
    for (int c = 1; c < nc; ++c)
        if (L.chips[c].tiles > L.chips[biggest].tiles) biggest = c;
    std::vector<int> all(static_cast<size_t>(kCtrlInts) * nc, 0), tail(static_cast<size_t>(kCtrlInts) * nc, 0);
    for (int c = 0; c < nc; ++c)
        if (c != biggest) tail[static_cast<size_t>(c) * kCtrlInts + kConverged] = 1;
    int *ctrl_d = reinterpret_cast<int *>(base + L.off_ctrl);
    hipEvent_t a = nullptr, b = nullptr;
    BKO_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(hipErrorOutOfMemory, "hipEventCreate");
    }
    bko_status rc = BKO_OK;
    float total = 0.f;
    for (const std::vector<int> *ctrl : {&all, &tail}) {
        if (hipMemcpyAsync(ctrl_d, ctrl->data(), sizeof(int) * ctrl->size(), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = hip_fail(hipErrorUnknown, "hipMemcpyAsync");
            break;
        }
        auto pass = [&]() -> bko_status {
            bko_status r;
            if ((r = launch_row<T>(0, x, 0)) != BKO_OK) return r;
            return launch_row<T>(1, x, 1);
        };
        if ((rc = pass()) != BKO_OK) break;
        constexpr int kReps = 5;
        (void)hipEventRecord(a, st);
        for (int r = 0; r < kReps && rc == BKO_OK; ++r) rc = pass();
        (void)hipEventRecord(b, st);
        const hipError_t e = hipEventSynchronize(b);
        if (rc != BKO_OK) break;
        if (e != hipSuccess) {
            rc = hip_fail(e, "hipEventSynchronize");
            break;
        }
        float t = 0.f;
        (void)hipEventElapsedTime(&t, a, b);
        total += t / kReps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ms = total;
    return rc;
}

}  // namespace

// Autotuner: choose how many row tiles each workgroup of the row kernels
// walks (which sets each chip's workgroup count and Gram-partial count) by
// timing every candidate on this batch and workspace, over the whole batch
// and over its largest chip alone.  The workspace contents are scratch here.
bko_status batch_tune(BatchPlan &p, void *work, hipStream_t st)
{
    const int nc = static_cast<int>(p.ops.size());
    const Layout L0 = make_layout(p.ops.data(), nc, p.s, p.compute, 1);
    if (row_kernel_lds(p.s, p.compute) > device_max_lds()) {
        set_error("s = %d needs %zu bytes of LDS per workgroup in this precision; the device grants %zu", p.s,
                  row_kernel_lds(p.s, p.compute), device_max_lds());
        return BKO_EINVAL;
    }
    bko_status rc;
    // finite, defined contents for the timed kernels
    if ((rc = launch_zero(work, L0.bytes, st)) != BKO_OK) return rc;
    p.tune_ms.clear();
    float best = 0.f;
    int best_tpw = 1;
    for (int tpw : {1, 2, 4, 8}) {
        float ms = 0.f;
        rc = p.compute == BKO_F64 ? time_granularity<double>(p, tpw, work, st, ms)
                                  : time_granularity<float>(p, tpw, work, st, ms);
        if (rc != BKO_OK) return rc;
        p.tune_ms.push_back({tpw, ms});
        if (p.tune_ms.size() == 1 || ms < best) {
            best = ms;
            best_tpw = tpw;
        }
    }
    p.tiles_per_wg = best_tpw;
    p.tuned = true;
    p.graphs.clear();
    return BKO_OK;
}

bko_status batch_solve(BatchPlan &p, const double *const *B, const int64_t *ldb, double *const *X, const int64_t *ldx,
                       const double *const *X0, const int64_t *ldx0, double tol, int max_iter, void *work,
                       bko_solve_info *infos, hipStream_t st)
{
    bko_status rc;
    if (!p.tuned && (rc = batch_tune(p, work, st)) != BKO_OK) return rc;
    const int nc = static_cast<int>(p.ops.size());
    const Layout L = make_layout(p.ops.data(), nc, p.s, p.compute, p.tiles_per_wg);
    if (p.compute == BKO_F64)
        return batch_solve_t<double>(L, work, B, ldb, X, ldx, X0, ldx0, tol, max_iter, infos, st, &p.graphs);
    return batch_solve_t<float>(L, work, B, ldb, X, ldx, X0, ldx0, tol, max_iter, infos, st, &p.graphs);
}

}  // namespace bko
