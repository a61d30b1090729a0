// Matrix-free variable-coefficient 5/7-point stencil over blocks of fields:
// Y[:, c] = A X[:, c]  (operator action, Sec. III-C, Eq. (6), and the block
// product inside the block solve, Sec. III-A), or Y = B - A X (residual).
//
// A is stored as its diagonal and the three forward-face couplings of every
// cell (wx[a] couples a with a+1, wy[a] with a+nx, wz[a] with a+nx*ny; zero
// where the neighbour is outside the grid), so
//   (A x)_a = diag_a x_a - wx_a x_{a+1} - wx_{a-1} x_{a-1}
//                        - wy_a x_{a+nx} - wy_{a-nx} x_{a-nx}
//                        - wz_a x_{a+p} - wz_{a-p} x_{a-p},     p = nx*ny.
//
// Two kernels.  stencil_tile_kernel (the operator action over many fields):
// full-width row tiles marched through z with the planes in LDS (a ring of
// three for BF16/FP32 planes) and 16-byte vector access; stencil_kernel (short tiles, unaligned views, the
// FP64 residual): a workgroup owns 256 consecutive cells and a group of
// columns, each thread loading its cell's seven coefficients once for every
// column of the group.  Both remap the workgroup order so that each XCD walks
// a contiguous range of work.  The damped Jacobi sweep that smooths an
// initial guess is the per-cell form with an update.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

constexpr int kThreads = 256;

template <class Tin, class Tout, class Tc, class Acc, bool kResidual>
__global__ __launch_bounds__(kThreads) void stencil_kernel(
    const Tc *__restrict__ diag, const Tc *__restrict__ wx, const Tc *__restrict__ wy,
    const Tc *__restrict__ wz, int nx, int ny, int nz, const Tin *__restrict__ X, int64_t ldx,
    Tout *__restrict__ Y, int64_t ldy, const double *__restrict__ Bres, int64_t ldb, int m,
    int cols_per_group, uint32_t ntiles, uint32_t nblocks, const int *__restrict__ skip, int *stop)
{
    if (skip && *skip) {
        // the iteration before this one converged: tell the later kernels
        if (stop && blockIdx.x == 0 && threadIdx.x == 0) *stop = 1;
        return;
    }
    const uint32_t lb = remap_block(blockIdx.x, nblocks);
    const uint32_t tile = lb % ntiles;
    const uint32_t group = lb / ntiles;
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int64_t n = plane * nz;
    const int64_t a = static_cast<int64_t>(tile) * kThreads + threadIdx.x;
    if (a >= n) return;
    const int i = static_cast<int>(a % nx);
    const int64_t q = a / nx;
    const int j = static_cast<int>(q % ny);
    const int l = static_cast<int>(q / ny);

    // neighbour offsets; a missing neighbour reads the cell itself with a
    // zero coupling so every load stays inside the column
    const int64_t oxm = i > 0 ? -1 : 0, oxp = i < nx - 1 ? 1 : 0;
    const int64_t oym = j > 0 ? -static_cast<int64_t>(nx) : 0, oyp = j < ny - 1 ? nx : 0;
    const int64_t ozm = l > 0 ? -plane : 0, ozp = l < nz - 1 ? plane : 0;
    const Acc d = static_cast<Acc>(diag[a]);
    const Acc cxp = static_cast<Acc>(wx[a]);
    const Acc cxm = i > 0 ? static_cast<Acc>(wx[a - 1]) : Acc(0);
    const Acc cyp = static_cast<Acc>(wy[a]);
    const Acc cym = j > 0 ? static_cast<Acc>(wy[a - nx]) : Acc(0);
    const Acc czp = static_cast<Acc>(wz[a]);
    const Acc czm = l > 0 ? static_cast<Acc>(wz[a - plane]) : Acc(0);

    const int c0 = static_cast<int>(group) * cols_per_group;
    const int c1 = min(m, c0 + cols_per_group);
    for (int c = c0; c < c1; ++c) {
        const Tin *x = X + static_cast<int64_t>(c) * ldx + a;
        const Acc xc = load_as<Acc>(x);
        const Acc nb = cxm * load_as<Acc>(x + oxm) + cxp * load_as<Acc>(x + oxp) +
                       cym * load_as<Acc>(x + oym) + cyp * load_as<Acc>(x + oyp) +
                       czm * load_as<Acc>(x + ozm) + czp * load_as<Acc>(x + ozp);
        Acc y = d * xc - nb;
        if constexpr (kResidual) y = static_cast<Acc>(Bres[static_cast<int64_t>(c) * ldb + a]) - y;
        Y[static_cast<int64_t>(c) * ldy + a] = store_from<Tout, Acc>(y);
    }
}

// ---------------------------------------------------------------- LDS-tiled kernel

// N consecutive elements moved with the widest aligned accesses.
template <class T, int N>
struct alignas(N * sizeof(T) >= 16 ? 16 : N * sizeof(T)) Vec {
    T v[N];
};

template <class T, int N>
__device__ __forceinline__ Vec<T, N> vload(const T *p)
{
    Vec<T, N> r;
    constexpr int B = N * sizeof(T);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int c = 0; c < B / 16; ++c) reinterpret_cast<uint4 *>(&r)[c] = reinterpret_cast<const uint4 *>(p)[c];
    } else if constexpr (B == 8) {
        *reinterpret_cast<uint2 *>(&r) = *reinterpret_cast<const uint2 *>(p);
    } else if constexpr (B == 4) {
        *reinterpret_cast<uint32_t *>(&r) = *reinterpret_cast<const uint32_t *>(p);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) r.v[i] = p[i];
    }
    return r;
}

template <class T, int N>
__device__ __forceinline__ void vstore(T *p, const Vec<T, N> &r)
{
    constexpr int B = N * sizeof(T);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int c = 0; c < B / 16; ++c) reinterpret_cast<uint4 *>(p)[c] = reinterpret_cast<const uint4 *>(&r)[c];
    } else if constexpr (B == 8) {
        *reinterpret_cast<uint2 *>(p) = *reinterpret_cast<const uint2 *>(&r);
    } else if constexpr (B == 4) {
        *reinterpret_cast<uint32_t *>(p) = *reinterpret_cast<const uint32_t *>(&r);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) p[i] = r.v[i];
    }
}

// Planes of the tile kept in LDS: a ring of three (this plane, the next,
// the one after) when the plane's LDS type is narrower than 8 bytes, else two
// (double-buffered; three FP64 planes would hold the kernel to two
// workgroups per CU, measured slower); ls = bytes of the LDS type.
__host__ __device__ constexpr int lds_planes(int ls) { return ls < 8 ? 3 : 2; }

// 16-byte vectors per thread and plane: as many as keep each of the plane
// arrays carried in registers (previous, current, next plane and the
// coupling below) at 64 bytes of accumulator values per thread, between one
// and four (FP64 or FP32 fields: four; BF16 fields with FP32 accumulation:
// two; more would hold the kernel to one wave per SIMD)
__host__ __device__ constexpr int tile_vecs(int vx, int acc_bytes)
{
    return 64 / (vx * acc_bytes) < 1 ? 1 : (64 / (vx * acc_bytes) > 4 ? 4 : 64 / (vx * acc_bytes));
}

// A workgroup owns full-width rows [j0, j0 + TY) of one field and marches
// through the nz planes with one barrier per plane.  FP64 planes: the
// current plane of the tile plus one halo row on each side sits in LDS
// (double-buffered), the planes below and above in registers.  Narrower
// planes: a ring of three planes with their halo rows in LDS (below).  Every
// global access of
// the field is a 16-byte vector access of consecutive cells.  Workgroups are
// ordered field-fastest within a tile and each XCD walks a contiguous range,
// so the coefficients of a tile (as many bytes per cell as the field itself,
// or twice as many) are read from HBM about once and served from that XCD's
// L2 to every field.
//
// The body takes the workgroup's logical index lb in [0, nblocks) of one
// operator's launch; stencil_tile_kernel runs one operator,
// stencil_tile_group_kernel the operators of a batch of chips in one grid.
template <class Tin, class Tout, class Tc, class Acc, bool kResidual>
__device__ __forceinline__ void stencil_tile_body(
    uint32_t lb, uint32_t nblocks, const Tc *__restrict__ diag, const Tc *__restrict__ wx,
    const Tc *__restrict__ wy, const Tc *__restrict__ wz, int nx, int ny, int nz, const Tin *__restrict__ X,
    int64_t ldx, Tout *__restrict__ Y, int64_t ldy, const double *__restrict__ Bres, int64_t ldb, int TY, int ntiles)
{
    constexpr int VX = 16 / sizeof(Tin);
    constexpr int R = tile_vecs(VX, sizeof(Acc));
    // fields fastest: the workgroups an XCD runs together share one tile's
    // coefficients (reused from L2); the halo rows of neighbouring tiles are
    // the only re-reads
    const uint32_t nf = nblocks / static_cast<uint32_t>(ntiles);
    const int tile = static_cast<int>(lb / nf);
    const int64_t field = lb % nf;
    const int j0 = tile * TY;
    const int rows = min(TY, ny - j0);
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int nvx = nx / VX;  // vectors per row
    const int nv = rows * nvx;
    extern __shared__ __align__(16) unsigned char smem[];
    // the LDS plane holds the narrower of the field's and the accumulator's
    // type (exact either way: a field value widened, or the value used), and
    // is written and read in whole VX-cell vectors
    using Ls = std::conditional_t<(sizeof(Tin) < sizeof(Acc)), Tin, Acc>;
    Ls *buf0 = reinterpret_cast<Ls *>(smem);
    const int bufsz = (TY + 2) * nx;
    const Tin *xf = X + field * ldx;
    Tout *yf = Y + field * ldy;
    const double *bf = kResidual ? Bres + field * ldb : nullptr;
    const int tid = threadIdx.x;

    int vrow[R], vx0[R];
    bool vok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = tid + r * kThreads;
        vok[r] = q < nv;
        vrow[r] = vok[r] ? q / nvx : 0;
        vx0[r] = vok[r] ? (q % nvx) * VX : 0;
    }
    // halo work: rows j0 - 1 and j0 + rows of the current plane
    const int hq = tid;  // < 2 * nvx handled by this thread
    const bool hok = hq < 2 * nvx;
    const int hside = hok ? hq / nvx : 0;
    const int hx0 = hok ? (hq % nvx) * VX : 0;
    const int hy = hside == 0 ? j0 - 1 : j0 + rows;
    const bool hin = hok && hy >= 0 && hy < ny;
    const int hlrow = hside == 0 ? 0 : rows + 1;

    if constexpr (lds_planes(sizeof(Ls)) == 3) {
        // Ring of three planes in LDS: the raw vectors of plane l + 2 (tile
        // and halo rows) are requested at the start of plane l and stored
        // into the ring at its end, so their HBM latency overlaps the work of
        // plane l; plane l and its upper neighbours are read from the ring,
        // the plane below from registers.  Slot (l + 2) % 3 held plane l - 1,
        // whose last readers finished before this plane's barrier.
        Vec<Tin, VX> raw[R], hraw;
        auto slot = [&](int l) { return buf0 + (l % 3) * bufsz; };
        auto fetch = [&](int l) __attribute__((always_inline)) {
            const int64_t pl = static_cast<int64_t>(l) * plane;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (vok[r] && l < nz) {
                    raw[r] = vload<Tin, VX>(xf + pl + static_cast<int64_t>(j0 + vrow[r]) * nx + vx0[r]);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e) raw[r].v[e] = Tin{};
                }
            }
            if (hin && l < nz) {
                hraw = vload<Tin, VX>(xf + pl + static_cast<int64_t>(hy) * nx + hx0);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) hraw.v[e] = Tin{};
            }
        };
        auto to_lds = [](const Vec<Tin, VX> &v) __attribute__((always_inline)) {
            if constexpr (std::is_same_v<Ls, Tin>) {
                return v;
            } else {
                Vec<Ls, VX> o;
#pragma unroll
                for (int e = 0; e < VX; ++e) o.v[e] = store_from<Ls, Acc>(load_as<Acc>(&v.v[e]));
                return o;
            }
        };
        auto stash = [&](int l) __attribute__((always_inline)) {
            Ls *b = slot(l);
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (vok[r]) vstore<Ls, VX>(b + (vrow[r] + 1) * nx + vx0[r], to_lds(raw[r]));
            if (hok) vstore<Ls, VX>(b + hlrow * nx + hx0, to_lds(hraw));
        };
        fetch(0);
        stash(0);
        fetch(1);
        stash(1);
        Acc prev[R][VX], wzm[R][VX];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                prev[r][e] = Acc(0);
                wzm[r][e] = Acc(0);
            }
        for (int l = 0; l < nz; ++l) {
            const int64_t pl = static_cast<int64_t>(l) * plane;
            fetch(l + 2);
            __syncthreads();
            const Ls *bc = slot(l), *bn = slot(l + 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!vok[r]) continue;
                const int j = j0 + vrow[r];
                const int64_t a = pl + static_cast<int64_t>(j) * nx + vx0[r];
                const Vec<Tc, VX> d = vload<Tc, VX>(diag + a);
                const Vec<Tc, VX> cx = vload<Tc, VX>(wx + a);
                const Vec<Tc, VX> cy = vload<Tc, VX>(wy + a);
                const Vec<Tc, VX> cz = vload<Tc, VX>(wz + a);
                Acc cym[VX];
                if (j > 0) {
                    const Vec<Tc, VX> t = vload<Tc, VX>(wy + a - nx);
#pragma unroll
                    for (int e = 0; e < VX; ++e) cym[e] = static_cast<Acc>(t.v[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e) cym[e] = Acc(0);
                }
                const Acc cxm0 = vx0[r] > 0 ? static_cast<Acc>(wx[a - 1]) : Acc(0);
                const int off = (vrow[r] + 1) * nx + vx0[r];
                const Ls *brow = bc + off;
                const Vec<Ls, VX> cv = vload<Ls, VX>(brow), nv = vload<Ls, VX>(bn + off);
                const Vec<Ls, VX> upv = vload<Ls, VX>(brow - nx), dnv = vload<Ls, VX>(brow + nx);
                const Acc left = vx0[r] > 0 ? load_as<Acc>(brow - 1) : Acc(0);
                const Acc right = vx0[r] + VX < nx ? load_as<Acc>(brow + VX) : Acc(0);
                Acc cur[VX];
#pragma unroll
                for (int e = 0; e < VX; ++e) cur[e] = load_as<Acc>(&cv.v[e]);
                Vec<Tout, VX> out;
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const Acc xm = e > 0 ? cur[e - 1] : left;
                    const Acc xp = e < VX - 1 ? cur[e + 1] : right;
                    const Acc cxm = e > 0 ? static_cast<Acc>(cx.v[e - 1]) : cxm0;
                    const Acc nb = cxm * xm + static_cast<Acc>(cx.v[e]) * xp + cym[e] * load_as<Acc>(&upv.v[e]) +
                                   static_cast<Acc>(cy.v[e]) * load_as<Acc>(&dnv.v[e]) + wzm[r][e] * prev[r][e] +
                                   static_cast<Acc>(cz.v[e]) * load_as<Acc>(&nv.v[e]);
                    Acc y = static_cast<Acc>(d.v[e]) * cur[e] - nb;
                    if constexpr (kResidual) y = static_cast<Acc>(bf[a + e]) - y;
                    out.v[e] = store_from<Tout, Acc>(y);
                    wzm[r][e] = static_cast<Acc>(cz.v[e]);
                    prev[r][e] = cur[e];
                }
                vstore<Tout, VX>(yf + a, out);
            }
            stash(l + 2);
        }
        return;
    }

    Acc prev[R][VX], cur[R][VX], nxt[R][VX], wzm[R][VX];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            prev[r][e] = Acc(0);
            wzm[r][e] = Acc(0);
            cur[r][e] = Acc(0);
        }
        if (vok[r]) {
            const Vec<Tin, VX> v = vload<Tin, VX>(xf + static_cast<int64_t>(j0 + vrow[r]) * nx + vx0[r]);
#pragma unroll
            for (int e = 0; e < VX; ++e) cur[r][e] = load_as<Acc>(&v.v[e]);
        }
    }

    for (int l = 0; l < nz; ++l) {
        const int64_t pl = static_cast<int64_t>(l) * plane;
        // prefetch the plane above
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int e = 0; e < VX; ++e) nxt[r][e] = Acc(0);
            if (vok[r] && l + 1 < nz) {
                const Vec<Tin, VX> v = vload<Tin, VX>(xf + pl + plane + static_cast<int64_t>(j0 + vrow[r]) * nx + vx0[r]);
#pragma unroll
                for (int e = 0; e < VX; ++e) nxt[r][e] = load_as<Acc>(&v.v[e]);
            }
        }
        // current plane of the tile into LDS, with the halo rows (zero outside the grid)
        Ls *buf = buf0 + (l & 1) * bufsz;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (vok[r]) {
                Vec<Ls, VX> v;
#pragma unroll
                for (int e = 0; e < VX; ++e) v.v[e] = store_from<Ls, Acc>(cur[r][e]);
                vstore<Ls, VX>(buf + (vrow[r] + 1) * nx + vx0[r], v);
            }
        }
        if (hok) {
            Vec<Ls, VX> hv;
            if (hin) {
                const Vec<Tin, VX> v = vload<Tin, VX>(xf + pl + static_cast<int64_t>(hy) * nx + hx0);
#pragma unroll
                for (int e = 0; e < VX; ++e) hv.v[e] = store_from<Ls, Acc>(load_as<Acc>(&v.v[e]));
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) hv.v[e] = store_from<Ls, Acc>(Acc(0));
            }
            vstore<Ls, VX>(buf + hlrow * nx + hx0, hv);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!vok[r]) continue;
            const int j = j0 + vrow[r];
            const int64_t a = pl + static_cast<int64_t>(j) * nx + vx0[r];
            const Vec<Tc, VX> d = vload<Tc, VX>(diag + a);
            const Vec<Tc, VX> cx = vload<Tc, VX>(wx + a);
            const Vec<Tc, VX> cy = vload<Tc, VX>(wy + a);
            const Vec<Tc, VX> cz = vload<Tc, VX>(wz + a);
            Acc cym[VX];
            if (j > 0) {
                const Vec<Tc, VX> t = vload<Tc, VX>(wy + a - nx);
#pragma unroll
                for (int e = 0; e < VX; ++e) cym[e] = static_cast<Acc>(t.v[e]);
            } else {
#pragma unroll
                for (int e = 0; e < VX; ++e) cym[e] = Acc(0);
            }
            const Acc cxm0 = vx0[r] > 0 ? static_cast<Acc>(wx[a - 1]) : Acc(0);
            const Ls *brow = buf + (vrow[r] + 1) * nx + vx0[r];
            const Acc left = vx0[r] > 0 ? load_as<Acc>(brow - 1) : Acc(0);
            const Acc right = vx0[r] + VX < nx ? load_as<Acc>(brow + VX) : Acc(0);
            const Vec<Ls, VX> upv = vload<Ls, VX>(brow - nx), dnv = vload<Ls, VX>(brow + nx);
            Vec<Tout, VX> out;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                const Acc xm = e > 0 ? cur[r][e - 1] : left;
                const Acc xp = e < VX - 1 ? cur[r][e + 1] : right;
                const Acc cxm = e > 0 ? static_cast<Acc>(cx.v[e - 1]) : cxm0;
                const Acc up = load_as<Acc>(&upv.v[e]);
                const Acc dn = load_as<Acc>(&dnv.v[e]);
                const Acc nb = cxm * xm + static_cast<Acc>(cx.v[e]) * xp + cym[e] * up +
                               static_cast<Acc>(cy.v[e]) * dn + wzm[r][e] * prev[r][e] +
                               static_cast<Acc>(cz.v[e]) * nxt[r][e];
                Acc y = static_cast<Acc>(d.v[e]) * cur[r][e] - nb;
                if constexpr (kResidual) y = static_cast<Acc>(bf[a + e]) - y;
                out.v[e] = store_from<Tout, Acc>(y);
                wzm[r][e] = static_cast<Acc>(cz.v[e]);
            }
            vstore<Tout, VX>(yf + a, out);
        }
        // roll the register planes
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                prev[r][e] = cur[r][e];
                cur[r][e] = nxt[r][e];
            }
    }
}

template <class Tin, class Tout, class Tc, class Acc, bool kResidual>
__global__ __launch_bounds__(kThreads) void stencil_tile_kernel(
    const Tc *__restrict__ diag, const Tc *__restrict__ wx, const Tc *__restrict__ wy, const Tc *__restrict__ wz,
    int nx, int ny, int nz, const Tin *__restrict__ X, int64_t ldx, Tout *__restrict__ Y, int64_t ldy,
    const double *__restrict__ Bres, int64_t ldb, int TY, int ntiles, uint32_t nblocks, const int *__restrict__ skip,
    int *stop)
{
    if (skip && *skip) {
        if (stop && blockIdx.x == 0 && threadIdx.x == 0) *stop = 1;
        return;
    }
    stencil_tile_body<Tin, Tout, Tc, Acc, kResidual>(remap_block(blockIdx.x, nblocks), nblocks, diag, wx, wy, wz, nx,
                                                     ny, nz, X, ldx, Y, ldy, Bres, ldb, TY, ntiles);
}

// One chip's share of a grouped operator action: workgroups
// [block0, block0 + ntiles * m) of the grid.
struct StencilJob {
    const void *diag, *wx, *wy, *wz;
    const void *X;
    void *Y;
    int64_t ldx, ldy;
    int nx, ny, nz, ty, ntiles, m;
    uint32_t block0;
    uint32_t pad;
};

// The operator action of every chip of a batch in one grid: each XCD walks
// a contiguous range of the (chip, tile, field) order; a workgroup finds
// its chip by binary search over the jobs' first blocks.
template <class Tin, class Tout, class Tc, class Acc>
__global__ __launch_bounds__(kThreads) void stencil_tile_group_kernel(const StencilJob *__restrict__ jobs, int njobs)
{
    const uint32_t g = remap_block(blockIdx.x, gridDim.x);
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].block0 <= g) lo = mid;
        else hi = mid - 1;
    }
    const StencilJob &j = jobs[lo];
    const uint32_t nb = static_cast<uint32_t>(j.ntiles) * static_cast<uint32_t>(j.m);
    stencil_tile_body<Tin, Tout, Tc, Acc, false>(
        g - j.block0, nb, static_cast<const Tc *>(j.diag), static_cast<const Tc *>(j.wx), static_cast<const Tc *>(j.wy),
        static_cast<const Tc *>(j.wz), j.nx, j.ny, j.nz, static_cast<const Tin *>(j.X), j.ldx, static_cast<Tout *>(j.Y),
        j.ldy, nullptr, 0, j.ty, j.ntiles);
}

// Tile height: about kThreads * VX * tile_vecs(VX) cells per plane, lowered until
// the launch has enough workgroups to fill the chip.
inline int tile_rows(int nx, int ny, int m, int vx, int acc_bytes)
{
    int ty = std::max(1, std::min(ny, kThreads * vx * tile_vecs(vx, acc_bytes) / nx));
    while (ty > 2 && static_cast<int64_t>((ny + ty - 1) / ty) * m < 2048) ty = (ty + 1) / 2;
    return ty;
}

// Rows per tile of stencil_tile_kernel for these fields, or 0 when the
// per-cell kernel takes them: rows not a whole number of 16-byte vectors,
// views not 16-byte aligned, or tiles too short to pay for their halo.
int tile_plan(const Operator &op, int m, size_t win, size_t wout, size_t wacc, uintptr_t X, int64_t ldx, uintptr_t Y,
              int64_t ldy)
{
    const int vx = static_cast<int>(16 / win);
    const size_t ya = std::min<size_t>(16, vx * wout);
    // one halo vector per thread: two halo rows of nx / vx vectors each
    const bool aligned = op.nx % vx == 0 && 2 * (op.nx / vx) <= kThreads && X % 16 == 0 &&
                         (ldx * win) % 16 == 0 && Y % ya == 0 && (ldy * wout) % ya == 0;
    if (!aligned || m <= 0) return 0;
    const int ty = tile_rows(op.nx, op.ny, m, vx, static_cast<int>(wacc));
    // short tiles waste the halo and most threads: the per-cell kernel is
    // better there (e.g. the few-column products inside the block solve)
    if (!(ty >= 8 || ty == op.ny)) return 0;
    if (static_cast<int64_t>(ty) * op.nx > static_cast<int64_t>(kThreads) * vx * tile_vecs(vx, static_cast<int>(wacc)))
        return 0;
    const int ntiles = (op.ny + ty - 1) / ty;
    if (static_cast<uint64_t>(ntiles) * m > 0x7fffffffu) return 0;
    return ty;
}

template <class Tin, class Tout, class Tc, class Acc, bool kResidual>
bko_status run(const Operator &op, const Tc *diag, const Tc *wx, const Tc *wy, const Tc *wz, int m,
               const void *X, int64_t ldx, void *Y, int64_t ldy, const double *Bres, int64_t ldb,
               hipStream_t stream, const int *skip, int *stop)
{
    const int ty = tile_plan(op, m, sizeof(Tin), sizeof(Tout), sizeof(Acc), reinterpret_cast<uintptr_t>(X), ldx,
                             reinterpret_cast<uintptr_t>(Y), ldy);
    if (ty > 0) {
        const int ntiles = (op.ny + ty - 1) / ty;
        const uint64_t nb = static_cast<uint64_t>(ntiles) * m;
        const size_t ls = std::min(sizeof(Acc), sizeof(Tin));
        const size_t lds = lds_planes(static_cast<int>(ls)) * ls * static_cast<size_t>(ty + 2) * op.nx;
        hipLaunchKernelGGL((stencil_tile_kernel<Tin, Tout, Tc, Acc, kResidual>), dim3(static_cast<uint32_t>(nb)),
                           dim3(kThreads), lds, stream, diag, wx, wy, wz, op.nx, op.ny, op.nz,
                           static_cast<const Tin *>(X), ldx, static_cast<Tout *>(Y), ldy, Bres, ldb, ty, ntiles,
                           static_cast<uint32_t>(nb), skip, stop);
        BKO_HIP(hipGetLastError());
        return BKO_OK;
    }
    const uint32_t ntiles = static_cast<uint32_t>((op.n + kThreads - 1) / kThreads);
    // enough column groups to fill the chip, few enough that each thread
    // reuses its coefficients over several columns
    int cols = 8;
    if (static_cast<int64_t>(ntiles) * ((m + cols - 1) / cols) < 4096) cols = 1;
    const uint32_t ngroups = static_cast<uint32_t>((m + cols - 1) / cols);
    const uint64_t nb = static_cast<uint64_t>(ntiles) * ngroups;
    if (nb > 0x7fffffffu) {
        set_error("stencil grid of %llu workgroups too large", (unsigned long long)nb);
        return BKO_EINVAL;
    }
    hipLaunchKernelGGL((stencil_kernel<Tin, Tout, Tc, Acc, kResidual>), dim3(static_cast<uint32_t>(nb)),
                       dim3(kThreads), 0, stream, diag, wx, wy, wz, op.nx, op.ny, op.nz,
                       static_cast<const Tin *>(X), ldx, static_cast<Tout *>(Y), ldy, Bres, ldb, m, cols,
                       ntiles, static_cast<uint32_t>(nb), skip, stop);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class Tin, class Tout>
bko_status dispatch_compute(const Operator &op, int m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                            bko_dtype compute, hipStream_t stream, const int *skip, int *stop)
{
    if (compute == BKO_F64)
        return run<Tin, Tout, double, double, false>(op, op.diag64, op.wx64, op.wy64, op.wz64, m, X, ldx, Y,
                                                     ldy, nullptr, 0, stream, skip, stop);
    return run<Tin, Tout, float, float, false>(op, op.diag32, op.wx32, op.wy32, op.wz32, m, X, ldx, Y, ldy,
                                               nullptr, 0, stream, skip, stop);
}

// One damped Jacobi sweep Y = X + omega (B - A X) / diag(A) (FP64), the
// smoother applied to an initial guess before the block solve.
__global__ __launch_bounds__(kThreads) void jacobi_kernel(const double *__restrict__ diag, const double *__restrict__ wx,
                                                          const double *__restrict__ wy, const double *__restrict__ wz,
                                                          int nx, int ny, int nz, const double *__restrict__ X,
                                                          int64_t ldx, const double *__restrict__ B, int64_t ldb,
                                                          double *__restrict__ Y, int64_t ldy, int m, double omega)
{
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int64_t n = plane * nz;
    const int64_t a = static_cast<int64_t>(remap_block(blockIdx.x, gridDim.x)) * kThreads + threadIdx.x;
    if (a >= n) return;
    const int i = static_cast<int>(a % nx);
    const int64_t q = a / nx;
    const int j = static_cast<int>(q % ny);
    const int l = static_cast<int>(q / ny);
    const int64_t oxm = i > 0 ? -1 : 0, oxp = i < nx - 1 ? 1 : 0;
    const int64_t oym = j > 0 ? -static_cast<int64_t>(nx) : 0, oyp = j < ny - 1 ? nx : 0;
    const int64_t ozm = l > 0 ? -plane : 0, ozp = l < nz - 1 ? plane : 0;
    const double d = diag[a];
    const double cxp = wx[a], cxm = i > 0 ? wx[a - 1] : 0.0;
    const double cyp = wy[a], cym = j > 0 ? wy[a - nx] : 0.0;
    const double czp = wz[a], czm = l > 0 ? wz[a - plane] : 0.0;
    const double sc = omega / d;
    for (int c = 0; c < m; ++c) {
        const double *x = X + c * ldx + a;
        const double nb = cxm * x[oxm] + cxp * x[oxp] + cym * x[oym] + cyp * x[oyp] + czm * x[ozm] + czp * x[ozp];
        const double r = B[c * ldb + a] - (d * x[0] - nb);
        Y[c * ldy + a] = fma(sc, r, x[0]);
    }
}

template <class Tin>
bko_status dispatch_out(const Operator &op, int m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                        bko_dtype t_out, bko_dtype compute, hipStream_t stream, const int *skip, int *stop)
{
    switch (t_out) {
    case BKO_F64: return dispatch_compute<Tin, double>(op, m, X, ldx, Y, ldy, compute, stream, skip, stop);
    case BKO_F32: return dispatch_compute<Tin, float>(op, m, X, ldx, Y, ldy, compute, stream, skip, stop);
    default: return dispatch_compute<Tin, bf16>(op, m, X, ldx, Y, ldy, compute, stream, skip, stop);
    }
}

template <class Tin, class Tout, class Tc, class Acc>
bko_status run_group(const std::vector<StencilJob> &jobs, uint32_t total, size_t lds, const void *jobs_dev,
                     hipStream_t stream)
{
    hipLaunchKernelGGL((stencil_tile_group_kernel<Tin, Tout, Tc, Acc>), dim3(total), dim3(kThreads), lds, stream,
                       static_cast<const StencilJob *>(jobs_dev), static_cast<int>(jobs.size()));
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class Tin, class Tout>
bko_status group_by_compute(const std::vector<StencilJob> &jobs, uint32_t total, size_t lds, const void *jobs_dev,
                            bko_dtype compute, hipStream_t stream)
{
    if (compute == BKO_F64) return run_group<Tin, Tout, double, double>(jobs, total, lds, jobs_dev, stream);
    return run_group<Tin, Tout, float, float>(jobs, total, lds, jobs_dev, stream);
}

template <class Tin>
bko_status group_by_out(const std::vector<StencilJob> &jobs, uint32_t total, size_t lds, const void *jobs_dev,
                        bko_dtype t_out, bko_dtype compute, hipStream_t stream)
{
    switch (t_out) {
    case BKO_F64: return group_by_compute<Tin, double>(jobs, total, lds, jobs_dev, compute, stream);
    case BKO_F32: return group_by_compute<Tin, float>(jobs, total, lds, jobs_dev, compute, stream);
    default: return group_by_compute<Tin, bf16>(jobs, total, lds, jobs_dev, compute, stream);
    }
}

}  // namespace

bko_status launch_stencil(const Operator &op, int m, const void *X, int64_t ldx, bko_dtype t_in, void *Y,
                          int64_t ldy, bko_dtype t_out, bko_dtype compute, const double *Bres, int64_t ldb,
                          hipStream_t stream, const int *skip, int *stop)
{
    if (m <= 0) return BKO_OK;
    if (Bres != nullptr) {
        // residual form is FP64 only
        return run<double, double, double, double, true>(op, op.diag64, op.wx64, op.wy64, op.wz64, m, X, ldx, Y,
                                                         ldy, Bres, ldb, stream, skip, stop);
    }
    switch (t_in) {
    case BKO_F64: return dispatch_out<double>(op, m, X, ldx, Y, ldy, t_out, compute, stream, skip, stop);
    case BKO_F32: return dispatch_out<float>(op, m, X, ldx, Y, ldy, t_out, compute, stream, skip, stop);
    default: return dispatch_out<bf16>(op, m, X, ldx, Y, ldy, t_out, compute, stream, skip, stop);
    }
}

size_t stencil_group_job_bytes(int nchips) { return sizeof(StencilJob) * static_cast<size_t>(nchips); }

bko_status launch_stencil_group(const Operator *const *ops, int nchips, const int *m, const void *const *X,
                                const int64_t *ldx, bko_dtype t_in, void *const *Y, const int64_t *ldy,
                                bko_dtype t_out, bko_dtype compute, int ty_cap, void *jobs_dev,
                                std::vector<unsigned char> &host_jobs, hipStream_t stream)
{
    const size_t win = dtype_size(t_in), wout = dtype_size(t_out);
    const size_t wacc = compute == BKO_F64 ? sizeof(double) : sizeof(float);
    const int vx = static_cast<int>(16 / win);
    const size_t ya = std::min<size_t>(16, vx * wout);
    const size_t ls = std::min(win, compute == BKO_F64 ? sizeof(double) : sizeof(float));
    std::vector<StencilJob> jobs;
    std::vector<int> rest;
    uint64_t total = 0;
    size_t lds = 0;
    for (int c = 0; c < nchips; ++c) {
        if (m[c] <= 0) continue;
        const Operator &op = *ops[c];
        const uintptr_t xa = reinterpret_cast<uintptr_t>(X[c]), ya_p = reinterpret_cast<uintptr_t>(Y[c]);
        const bool aligned = op.nx % vx == 0 && 2 * (op.nx / vx) <= kThreads && xa % 16 == 0 &&
                             (ldx[c] * win) % 16 == 0 && ya_p % ya == 0 && (ldy[c] * wout) % ya == 0;
        if (!aligned) {
            rest.push_back(c);
            continue;
        }
        // the batch fills the chip: full-height tiles of about kThreads * vx
        // * tile_vecs(vx) cells per plane (or at most ty_cap rows)
        int ty = std::max(1, std::min(op.ny, kThreads * vx * tile_vecs(vx, static_cast<int>(wacc)) / op.nx));
        if (ty_cap > 0) ty = std::min(ty, ty_cap);
        StencilJob j{};
        const bool f64 = compute == BKO_F64;
        j.diag = f64 ? static_cast<const void *>(op.diag64) : static_cast<const void *>(op.diag32);
        j.wx = f64 ? static_cast<const void *>(op.wx64) : static_cast<const void *>(op.wx32);
        j.wy = f64 ? static_cast<const void *>(op.wy64) : static_cast<const void *>(op.wy32);
        j.wz = f64 ? static_cast<const void *>(op.wz64) : static_cast<const void *>(op.wz32);
        j.X = X[c];
        j.Y = Y[c];
        j.ldx = ldx[c];
        j.ldy = ldy[c];
        j.nx = op.nx;
        j.ny = op.ny;
        j.nz = op.nz;
        j.ty = ty;
        j.ntiles = (op.ny + ty - 1) / ty;
        j.m = m[c];
        j.block0 = static_cast<uint32_t>(total);
        total += static_cast<uint64_t>(j.ntiles) * m[c];
        lds = std::max(lds, lds_planes(static_cast<int>(ls)) * ls * static_cast<size_t>(ty + 2) * op.nx);
        jobs.push_back(j);
    }
    if (total > 0x7fffffffu) {
        set_error("grouped operator action of %llu workgroups too large", (unsigned long long)total);
        return BKO_EINVAL;
    }
    bko_status rc = BKO_OK;
    if (!jobs.empty()) {
        const size_t bytes = sizeof(StencilJob) * jobs.size();
        host_jobs.resize(bytes);
        std::memcpy(host_jobs.data(), jobs.data(), bytes);
        BKO_HIP(hipMemcpyAsync(jobs_dev, host_jobs.data(), bytes, hipMemcpyHostToDevice, stream));
        const uint32_t tot = static_cast<uint32_t>(total);
        switch (t_in) {
        case BKO_F64: rc = group_by_out<double>(jobs, tot, lds, jobs_dev, t_out, compute, stream); break;
        case BKO_F32: rc = group_by_out<float>(jobs, tot, lds, jobs_dev, t_out, compute, stream); break;
        default: rc = group_by_out<bf16>(jobs, tot, lds, jobs_dev, t_out, compute, stream); break;
        }
        if (rc != BKO_OK) return rc;
    }
    // chips whose rows or views do not suit the tiled kernel: one launch each
    for (int c : rest)
        if ((rc = launch_stencil(*ops[c], m[c], X[c], ldx[c], t_in, Y[c], ldy[c], t_out, compute, nullptr, 0, stream)) !=
            BKO_OK)
            return rc;
    return BKO_OK;
}

int stencil_tile_rows(const Operator &op, int m, const void *X, int64_t ldx, bko_dtype t_in, const void *Y,
                      int64_t ldy, bko_dtype t_out, bko_dtype compute)
{
    return tile_plan(op, m, dtype_size(t_in), dtype_size(t_out), compute == BKO_F64 ? sizeof(double) : sizeof(float),
                     reinterpret_cast<uintptr_t>(X), ldx, reinterpret_cast<uintptr_t>(Y), ldy);
}

bko_status launch_jacobi(const Operator &op, int m, const double *B, int64_t ldb, double *X, int64_t ldx,
                         double *work, int64_t ldw, int sweeps, double omega, hipStream_t stream)
{
    if (m <= 0 || sweeps <= 0) return BKO_OK;
    const unsigned blocks = static_cast<unsigned>((op.n + kThreads - 1) / kThreads);
    const double *src = X;
    int64_t lds = ldx;
    for (int k = 0; k < sweeps; ++k) {
        // even sweeps write the work block, odd sweeps write X back
        double *dst = (k % 2 == 0) ? work : X;
        const int64_t ldd = (k % 2 == 0) ? ldw : ldx;
        hipLaunchKernelGGL(jacobi_kernel, dim3(blocks), dim3(kThreads), 0, stream, op.diag64, op.wx64, op.wy64, op.wz64,
                           op.nx, op.ny, op.nz, src, lds, B, ldb, dst, ldd, m, omega);
        BKO_HIP(hipGetLastError());
        src = dst;
        lds = ldd;
    }
    if (sweeps % 2 == 1) {
        // the last sweep landed in the work block: one more plain copy
        BKO_HIP(hipMemcpy2DAsync(X, sizeof(double) * ldx, work, sizeof(double) * ldw, sizeof(double) * op.n, m,
                                 hipMemcpyDeviceToDevice, stream));
    }
    return BKO_OK;
}

}  // namespace bko
