// Combination of basis solutions into temperature fields, T = X C
// (Sec. III-B, Eq. (5)): an n x s by s x m product with a short inner
// dimension (s <= 64), so the kernel is bound by the store of T.
//
// Each workgroup owns a 64-cell tile of X, kept in registers as matrix-core
// operands for the whole launch, and walks a range of fields 64 at a time:
// stage the 64-field slice of C in LDS, run the 16x16 matrix-core products
// (one 16-cell row block per wave, four 16-field blocks), stage the 64 x 64
// output tile in LDS and write it back with 16-byte coalesced stores.
//
// Modes: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32, FP32
// accumulate) and BF16 (inputs rounded to BF16, v_mfma_f32_16x16x32_bf16,
// FP32 accumulate).  Matrix-core operand layout for the 16x16 shapes: lane
// L supplies A[L % 16][k] and B[k][L % 16] for the k slot(s) of lane group
// L / 16; its four results are D[mfma_row(L / 16, r)][L % 16] (see
// common.hpp: the FP64 shape interleaves the rows).
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kTM = 64;       // cells per workgroup tile
constexpr int kTN = 64;       // fields per inner step
constexpr int kThreads = 256; // four waves

enum Mode { kF64 = 0, kF32 = 1, kBF16 = 2 };

template <int M> struct ModeTraits;
template <> struct ModeTraits<kF64> {
    using Acc = double;
    using Stage = double;  // C slice element in LDS
    static constexpr int kK = 4;
};
template <> struct ModeTraits<kF32> {
    using Acc = float;
    using Stage = float;
    static constexpr int kK = 4;
};
template <> struct ModeTraits<kBF16> {
    using Acc = float;
    using Stage = uint16_t;
    static constexpr int kK = 32;
};

__device__ inline __bf16 bits_to_bf(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

template <int kMode, class Tx, class Tc, class Tt>
__device__ __forceinline__ void combine_body(uint32_t bid, int64_t n, int s, int64_t m, const Tx *__restrict__ X,
                                             int64_t ldx, const Tc *__restrict__ C, int64_t ldc, Tt *__restrict__ T,
                                             int64_t ldt, int64_t fields_per_wg, uint32_t ntiles, int vec_ok)
{
    using TR = ModeTraits<kMode>;
    using Acc = typename TR::Acc;
    using Stage = typename TR::Stage;
    constexpr int kK = TR::kK;
    constexpr int kMaxSteps = 64 / kK;  // s <= 64

    const int ksteps = (s + kK - 1) / kK;
    const int s_pad = ksteps * kK;
    // LDS: the C slice [kTN][cstride], then (aliasing it once the matrix-core
    // products are done) the output tile [kTN][ostride]
    const int cstride = kMode == kBF16 ? s_pad + 8 : s_pad + 1;
    constexpr int ostride = kTM + (sizeof(Acc) == 8 ? 2 : 4);
    extern __shared__ __align__(16) unsigned char smem[];
    Stage *Cs = reinterpret_cast<Stage *>(smem);
    Acc *Os = reinterpret_cast<Acc *>(smem);

    const uint32_t tile = bid % ntiles;
    const uint32_t split = bid / ntiles;
    const int64_t cell0 = static_cast<int64_t>(tile) * kTM;
    const int64_t f_begin = static_cast<int64_t>(split) * fields_per_wg;
    const int64_t f_end = min(m, f_begin + fields_per_wg);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int li = lane & 15;  // row (cell) / column (field) within a 16-block
    const int lg = lane >> 4;  // k group

    // ---- A operands: the wave's 16 cells of X over all k, kept in registers
    const int64_t my_cell = cell0 + wave * 16 + li;
    const bool cell_ok = my_cell < n;
    double a64[kMode == kF64 ? kMaxSteps : 1];
    float a32[kMode == kF32 ? kMaxSteps : 1];
    bf8 abf[kMode == kBF16 ? kMaxSteps : 1];
#pragma unroll
    for (int t = 0; t < kMaxSteps; ++t) {
        if (t < ksteps) {
            if constexpr (kMode == kBF16) {
                bf8 v;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = t * kK + lg * 8 + e;
                    const float x = (cell_ok && k < s) ? load_as<float>(X + static_cast<int64_t>(k) * ldx + my_cell) : 0.f;
                    v[e] = bits_to_bf(f32_to_bf16(x));
                }
                abf[t] = v;
            } else {
                const int k = t * kK + lg;
                const Acc x = (cell_ok && k < s) ? load_as<Acc>(X + static_cast<int64_t>(k) * ldx + my_cell) : Acc(0);
                if constexpr (kMode == kF64) a64[t] = x;
                else a32[t] = x;
            }
        }
    }

    constexpr int kVec = 16 / sizeof(Tt);
    for (int64_t fb = f_begin; fb < f_end; fb += kTN) {
        __syncthreads();  // previous tile's LDS reads are done
        // ---- stage C[0:s_pad, fb:fb+64] as Cs[f][k]
        for (int idx = tid; idx < kTN * s_pad; idx += kThreads) {
            const int f = idx / s_pad;
            const int k = idx - f * s_pad;
            const int64_t field = fb + f;
            Stage v;
            if constexpr (kMode == kBF16) {
                const float c = (k < s && field < m) ? load_as<float>(C + field * ldc + k) : 0.f;
                v = f32_to_bf16(c);
            } else {
                v = (k < s && field < m) ? load_as<Acc>(C + field * ldc + k) : Acc(0);
            }
            Cs[f * cstride + k] = v;
        }
        __syncthreads();
        // ---- four 16x16 blocks per wave, accumulators kept in registers
        using AccV = typename std::conditional<kMode == kF64, d4, f4>::type;
        AccV acc[kTN / 16];
#pragma unroll
        for (int jb = 0; jb < kTN / 16; ++jb) {
            const Stage *cb = Cs + (jb * 16 + li) * cstride;
            acc[jb] = AccV{0, 0, 0, 0};
            if constexpr (kMode == kF64) {
#pragma unroll
                for (int t = 0; t < kMaxSteps; ++t)
                    if (t < ksteps) acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a64[t], cb[t * kK + lg], acc[jb], 0, 0, 0);
            } else if constexpr (kMode == kF32) {
#pragma unroll
                for (int t = 0; t < kMaxSteps; ++t)
                    if (t < ksteps) acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[t], cb[t * kK + lg], acc[jb], 0, 0, 0);
            } else {
#pragma unroll
                for (int t = 0; t < kMaxSteps; ++t) {
                    if (t < ksteps) {
                        bf8 b;
#pragma unroll
                        for (int e = 0; e < 8; ++e) b[e] = bits_to_bf(cb[t * kK + lg * 8 + e]);
                        acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(abf[t], b, acc[jb], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();  // every wave is done with the C slice: reuse it for the output tile
#pragma unroll
        for (int jb = 0; jb < kTN / 16; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Os[(jb * 16 + li) * ostride + wave * 16 + mfma_row<kMode == kF64>(lg, r)] = acc[jb][r];
        __syncthreads();
        // ---- write the 64 x 64 tile: fields are columns of T
        constexpr int kVecPerField = kTM / kVec;
        for (int idx = tid; idx < kTN * kVecPerField; idx += kThreads) {
            const int f = idx / kVecPerField;
            const int cv = idx - f * kVecPerField;
            const int64_t field = fb + f;
            if (field >= m) continue;
            const int64_t cell = cell0 + cv * kVec;
            Tt *dst = T + field * ldt + cell;
            const Acc *src = Os + f * ostride + cv * kVec;
            if (vec_ok && cell + kVec <= n) {
                union {
                    Tt e[kVec];
                    uint4 v;
                } u;
#pragma unroll
                for (int e = 0; e < kVec; ++e) u.e[e] = store_from<Tt, Acc>(src[e]);
                *reinterpret_cast<uint4 *>(dst) = u.v;
            } else {
                for (int e = 0; e < kVec && cell + e < n; ++e) dst[e] = store_from<Tt, Acc>(src[e]);
            }
        }
    }
}

template <int kMode, class Tx, class Tc, class Tt>
__global__ __launch_bounds__(kThreads) void combine_kernel(int64_t n, int s, int64_t m,
                                                           const Tx *__restrict__ X, int64_t ldx,
                                                           const Tc *__restrict__ C, int64_t ldc,
                                                           Tt *__restrict__ T, int64_t ldt,
                                                           int64_t fields_per_wg, uint32_t ntiles, int vec_ok)
{
    combine_body<kMode, Tx, Tc, Tt>(blockIdx.x, n, s, m, X, ldx, C, ldc, T, ldt, fields_per_wg, ntiles, vec_ok);
}

// One chip's share of a grouped combination: workgroups [block0, block0 +
// ntiles * splits) of the grid.
struct CombineJob {
    const double *X;
    const double *C;
    void *T;
    int64_t ldx, ldc, ldt, n, m, fields_per_wg;
    uint32_t ntiles, block0;
    int vec_ok, pad;
};

__device__ __forceinline__ const CombineJob &find_job(const CombineJob *__restrict__ jobs, int njobs, uint32_t g)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].block0 <= g) lo = mid;
        else hi = mid - 1;
    }
    return jobs[lo];
}

// The combination of every chip of a batch in one grid (FP32 / BF16 modes).
template <int kMode, class Tt>
__global__ __launch_bounds__(kThreads) void combine_group_kernel(const CombineJob *__restrict__ jobs, int njobs, int s)
{
    const CombineJob &j = find_job(jobs, njobs, blockIdx.x);
    combine_body<kMode, double, double, Tt>(blockIdx.x - j.block0, j.n, s, j.m, j.X, j.ldx, j.C, j.ldc,
                                            static_cast<Tt *>(j.T), j.ldt, j.fields_per_wg, j.ntiles, j.vec_ok);
}

// ---------------------------------------------------------------- wide BF16 tiles

// The BF16 combination with wide cell tiles, for BF16 or FP32 fields: a
// workgroup of eight waves owns 1024 consecutive cells (each wave 128 of
// them, as eight 16-cell blocks of matrix-core A operands rounded to BF16
// and held in registers for the whole launch).  C is rounded to BF16 and
// staged in LDS 128 fields at a time (one barrier per 128 fields; the next
// chunk is fetched into registers meanwhile); each wave then runs 16 fields
// at a time on v_mfma_f32_16x16x32_bf16 (FP32 accumulation), stages its own
// 16 x 128 results in a wave-private LDS slice and writes every field's 128
// cells (256 bytes for BF16 fields) with 16-byte stores, without waiting for
// the other waves.
constexpr int kWideWaves = 8;
constexpr int kWideThreads = 64 * kWideWaves;
constexpr int kWideRB = 8;                          // 16-cell blocks per wave
constexpr int kWideWC = kWideRB * 16;               // 128 cells per wave
constexpr int kWideTM = kWideWaves * kWideWC;       // 1024 cells per workgroup
constexpr int kWideF = 16;                          // fields per matrix-core block
constexpr int kWideChunk = 128;                     // fields per staged C chunk
constexpr int kWideCS = 64 + 8;                     // LDS row of C (BF16, padded)
constexpr int kWideOS = kWideWC + 8;                // LDS row of a wave's output slice (padded)

template <class Tx, class Tc, class Tt>
__global__ __launch_bounds__(kWideThreads) void combine_wide_kernel(int64_t n, int s, int64_t m,
                                                                    const Tx *__restrict__ X, int64_t ldx,
                                                                    const Tc *__restrict__ C, int64_t ldc,
                                                                    Tt *__restrict__ T, int64_t ldt,
                                                                    int64_t fields_per_wg, uint32_t ntiles, int vec_ok)
{
    const uint32_t tile = blockIdx.x % ntiles;
    const uint32_t split = blockIdx.x / ntiles;
    const int64_t cell0 = static_cast<int64_t>(tile) * kWideTM;
    const int64_t f_begin = static_cast<int64_t>(split) * fields_per_wg;
    const int64_t f_end = min(m, f_begin + fields_per_wg);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t wcell0 = cell0 + wave * kWideWC;
    __shared__ __align__(16) uint16_t cs[2][kWideChunk * kWideCS];
    __shared__ __align__(16) Tt os[kWideWaves][kWideF * kWideOS];
    Tt *myos = os[wave];

    // A operands: cell wcell0 + rb 16 + li, k = 32 t + 8 lg + e; every load
    // is issued (at a clamped index) and the padding zeroed afterwards, so
    // the loads are in flight together
    bf8 xa[kWideRB][2];
#pragma unroll
    for (int rb = 0; rb < kWideRB; ++rb) {
        const int64_t cell = wcell0 + rb * 16 + li;
        const int64_t cellc = cell < n ? cell : n - 1;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            bf8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 32 * t + 8 * lg + e;
                const int kc = k < s ? k : s - 1;
                const float x = load_as<float>(X + static_cast<int64_t>(kc) * ldx + cellc);
                v[e] = bits_to_bf(f32_to_bf16((k < s && cell < n) ? x : 0.f));
            }
            xa[rb][t] = v;
        }
    }
    // C chunk [128 fields][64 k] in BF16, 16 elements per thread, fetched
    // into registers one chunk ahead
    constexpr int kCE = kWideChunk * 64 / kWideThreads;
    uint16_t cv[kCE];
    auto fetch_c = [&](int64_t f0) {
#pragma unroll
        for (int i = 0; i < kCE; ++i) {
            const int e = tid + i * kWideThreads;
            const int f = e / 64, k = e % 64;
            const int64_t field = f0 + f;
            const int64_t fc = field < f_end ? field : f_end - 1;
            const int kc = k < s ? k : s - 1;
            const float c = load_as<float>(C + fc * ldc + kc);
            cv[i] = f32_to_bf16((k < s && field < f_end) ? c : 0.f);
        }
    };
    auto stash_c = [&](int b) {
#pragma unroll
        for (int i = 0; i < kCE; ++i) {
            const int e = tid + i * kWideThreads;
            cs[b][(e / 64) * kWideCS + e % 64] = cv[i];
        }
    };
    constexpr int kVec = 16 / sizeof(Tt);
    constexpr int kVPF = kWideWC / kVec;  // 16-byte vectors per field of the wave's slice
    if (f_begin < f_end) {
        fetch_c(f_begin);
        stash_c(0);
    }
    int b = 0;
    for (int64_t c0 = f_begin; c0 < f_end; c0 += kWideChunk) {
        const bool more = c0 + kWideChunk < f_end;
        if (more) fetch_c(c0 + kWideChunk);
        __syncthreads();  // chunk b staged; every wave is done with chunk b ^ 1
        const int64_t c1 = min(f_end, c0 + kWideChunk);
        for (int64_t f0 = c0; f0 < c1; f0 += kWideF) {
            const int fb = static_cast<int>(f0 - c0);
            bf8 cb[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                cb[t] = *reinterpret_cast<const bf8 *>(&cs[b][(fb + li) * kWideCS + 32 * t + 8 * lg]);
#pragma unroll
            for (int rb = 0; rb < kWideRB; ++rb) {
                // the second k step multiplies zeros when s <= 32
                f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[rb][0], cb[0], f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[rb][1], cb[1], acc, 0, 0, 0);
                // acc[r] = T[cell wcell0 + rb 16 + 4 lg + r][field f0 + li]:
                // four consecutive cells, one 8- or 16-byte LDS store
                Tt *dst = &myos[li * kWideOS + rb * 16 + 4 * lg];
                if constexpr (sizeof(Tt) == 2) {
                    uint2 pk;
                    pk.x = static_cast<uint32_t>(f32_to_bf16(acc[0])) | (static_cast<uint32_t>(f32_to_bf16(acc[1])) << 16);
                    pk.y = static_cast<uint32_t>(f32_to_bf16(acc[2])) | (static_cast<uint32_t>(f32_to_bf16(acc[3])) << 16);
                    *reinterpret_cast<uint2 *>(dst) = pk;
                } else {
                    *reinterpret_cast<float4 *>(dst) = make_float4(acc[0], acc[1], acc[2], acc[3]);
                }
            }
            // the slice is the wave's own: its lanes' stores are visible to
            // the wave once they have completed
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int q = 0; q < kWideF * kVPF / 64; ++q) {
                const int v = lane + q * 64;
                const int f = v / kVPF, cvi = v % kVPF;
                const int64_t field = f0 + f;
                const int64_t cell = wcell0 + static_cast<int64_t>(cvi) * kVec;
                if (field >= c1 || cell >= n) continue;
                const Tt *src = &myos[f * kWideOS + cvi * kVec];
                Tt *dst = T + field * ldt + cell;
                if (vec_ok && cell + kVec <= n) {
                    *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(src);
                } else {
                    for (int e = 0; e < kVec && cell + e < n; ++e) dst[e] = src[e];
                }
            }
            // the slice is rewritten by the next block only after every
            // lane has read it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (more) stash_c(b ^ 1);
        b ^= 1;
    }
}

// ---------------------------------------------------------------- noise

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): a counter-based generator, ten rounds of two
// 32 x 32 -> 64-bit products with the published multipliers and Weyl key
// increments.  The noise of field f (global index) at cell a is a pure
// function of (seed, f, a), so any split of the fields over calls or
// workgroups draws the same values.
struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// An open-interval uniform in (0, 1) from 52 random bits: (u + 1/2) 2^-52.
__device__ __forceinline__ double unit_open(uint32_t hi, uint32_t lo)
{
    const uint64_t u = (static_cast<uint64_t>(hi) << 20) | (lo >> 12);
    return (static_cast<double>(u) + 0.5) * 0x1.0p-52;
}

// Noise value of (field, cell): uniform on (-a, a) as a ((2u + 1) 2^-52 - 1)
// (exact before the product with a), or Gaussian N(0, a^2) by Box-Muller.
__device__ __forceinline__ double noise_value(int kind, double amp, uint64_t seed, uint64_t field, int64_t cell)
{
    const Philox4 r = philox4x32_10(static_cast<uint32_t>(cell), static_cast<uint32_t>(static_cast<uint64_t>(cell) >> 32),
                                    static_cast<uint32_t>(field), static_cast<uint32_t>(field >> 32),
                                    static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    if (kind == BKO_NOISE_UNIFORM) {
        const uint64_t u = (static_cast<uint64_t>(r.v[0]) << 20) | (r.v[1] >> 12);
        return amp * (static_cast<double>(2 * u + 1) * 0x1.0p-52 - 1.0);
    }
    const double x1 = unit_open(r.v[0], r.v[1]), x2 = unit_open(r.v[2], r.v[3]);
    return amp * (sqrt(-2.0 * log(x1)) * cos(6.283185307179586476925 * x2));
}

struct NoiseArgs {
    int kind;  // BKO_NOISE_*
    double amp;
    uint64_t seed, field_offset;
};

// E[f * lde + a] = noise of (field_offset + f, a)
__global__ __launch_bounds__(kThreads) void noise_fill_kernel(int64_t n, int64_t m, double *__restrict__ E, int64_t lde,
                                                              NoiseArgs na)
{
    const int64_t f = blockIdx.y;
    for (int64_t a = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; a < n;
         a += static_cast<int64_t>(gridDim.x) * kThreads)
        E[f * lde + a] = noise_value(na.kind, na.amp, na.seed, na.field_offset + f, a);
}

// alpha_j = mu_j / sum_k mu_kj per field j (C column j, ldc), summed in k
// order; a field whose |sum| < min_abs keeps its weights and gets flag 1.
__global__ __launch_bounds__(kThreads) void normalize_weights_kernel(int s, int64_t m, double *__restrict__ C, int64_t ldc,
                                                                     double min_abs, int *__restrict__ flags)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= m) return;
    double *c = C + j * ldc;
    double sum = 0.0;
    for (int k = 0; k < s; ++k) sum += c[k];
    const bool bad = !(fabs(sum) >= min_abs);
    flags[j] = bad ? 1 : 0;
    if (bad) return;
    for (int k = 0; k < s; ++k) c[k] = c[k] / sum;
}

// FP64 combination with direct stores, and its two-product form.
//
// The product is formed transposed, T^T tile = C^T X^T, so that the matrix
// core's result layout puts 16 consecutive cells of one field in the 16
// lanes of a lane group: every store instruction writes four full 128-byte
// lines of T, with no staging of the results.  Each wave owns 16 cells (its
// X rows stay in registers as the B operand); the A operand (C for 16
// fields) is staged once per workgroup in LDS by coalesced loads, double
// buffered, one barrier per 16 fields.  The k index
// of the contraction is laid out so that lane group g holds k = g KS .. g KS
// + KS - 1 (any bijection of k onto the MFMA slots gives the same sum).
// kDual: also F = Y C with Y = A X, the operator action of every field
// formed from the s columns of A X (Sec. III-C applied to Eq. (5)'s sum).
template <bool kDual, bool kNoise, int kMaxKS>
__device__ __forceinline__ void combine_direct_body(uint32_t bid, int64_t n, int s, int64_t m,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    const double *__restrict__ Y, int64_t ldy,
                                                    const double *__restrict__ C, int64_t ldc,
                                                    double *__restrict__ T, int64_t ldt, double *__restrict__ F,
                                                    int64_t ldf, int64_t fields_per_wg, uint32_t ntiles, NoiseArgs na)
{
    const int ks = (s + 3) / 4;  // <= kMaxKS
    const uint32_t tile = bid % ntiles;
    const uint32_t split = bid / ntiles;
    const int64_t f_begin = static_cast<int64_t>(split) * fields_per_wg;
    const int64_t f_end = min(m, f_begin + fields_per_wg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t cell = static_cast<int64_t>(tile) * kTM + wave * 16 + li;
    const bool cell_ok = cell < n;
    double xb[kMaxKS], yb[kDual ? kMaxKS : 1];
#pragma unroll
    for (int t = 0; t < kMaxKS; ++t) {
        const int k = lg * ks + t;
        const bool ok = t < ks && k < s && cell_ok;
        xb[t] = ok ? X[static_cast<int64_t>(k) * ldx + cell] : 0.0;
        if constexpr (kDual) yb[t] = ok ? Y[static_cast<int64_t>(k) * ldy + cell] : 0.0;
    }
    // 16 fields at a time: the workgroup stages C for the block in LDS
    // (coalesced loads, shared by its four waves), the next block's loads
    // in flight during this block's products and stores
    constexpr int kCS = 4 * kMaxKS + 1;                   // LDS row stride (padded)
    constexpr int kCR = (16 * 4 * kMaxKS + kThreads - 1) / kThreads;
    __shared__ double cbuf[2][16 * kCS];
    const int s4 = 4 * ks;
    double cv[kCR];
    auto fetch_c = [&](int64_t f0) {
#pragma unroll
        for (int i = 0; i < kCR; ++i) {
            const int e = threadIdx.x + i * kThreads;
            const int r = e / s4, k = e % s4;
            cv[i] = (e < 16 * s4 && k < s && f0 + r < f_end) ? C[(f0 + r) * ldc + k] : 0.0;
        }
    };
    auto stash_c = [&](int b) {
#pragma unroll
        for (int i = 0; i < kCR; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < 16 * s4) cbuf[b][(e / s4) * kCS + e % s4] = cv[i];
        }
    };
    if (f_begin < f_end) {
        fetch_c(f_begin);
        stash_c(0);
    }
    __syncthreads();
    int b = 0;
    for (int64_t f0 = f_begin; f0 < f_end; f0 += 16) {
        const bool more = f0 + 16 < f_end;
        if (more) fetch_c(f0 + 16);
        double a[kMaxKS];
#pragma unroll
        for (int t = 0; t < kMaxKS; ++t) a[t] = t < ks ? cbuf[b][li * kCS + lg * ks + t] : 0.0;
        d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < kMaxKS; ++t) {
            if (t < ks) {
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], xb[t], acc, 0, 0, 0);
                if constexpr (kDual) acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], yb[t], acc2, 0, 0, 0);
            }
        }
        if (cell_ok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t field = f0 + mfma_row<true>(lg, r);
                if (field < f_end) {
                    double t = acc[r];
                    if constexpr (kNoise) t += noise_value(na.kind, na.amp, na.seed, na.field_offset + field, cell);
                    T[field * ldt + cell] = t;
                    if constexpr (kDual) F[field * ldf + cell] = acc2[r];
                }
            }
        }
        if (more) stash_c(b ^ 1);
        __syncthreads();
        b ^= 1;
    }
}

template <bool kDual, bool kNoise, int kMaxKS>
__global__ __launch_bounds__(kThreads) void combine_direct_kernel(int64_t n, int s, int64_t m,
                                                                  const double *__restrict__ X, int64_t ldx,
                                                                  const double *__restrict__ Y, int64_t ldy,
                                                                  const double *__restrict__ C, int64_t ldc,
                                                                  double *__restrict__ T, int64_t ldt,
                                                                  double *__restrict__ F, int64_t ldf,
                                                                  int64_t fields_per_wg, uint32_t ntiles, NoiseArgs na)
{
    combine_direct_body<kDual, kNoise, kMaxKS>(blockIdx.x, n, s, m, X, ldx, Y, ldy, C, ldc, T, ldt, F, ldf,
                                               fields_per_wg, ntiles, na);
}

// The FP64 combination of every chip of a batch in one grid.
template <int kMaxKS>
__global__ __launch_bounds__(kThreads) void combine_direct_group_kernel(const CombineJob *__restrict__ jobs, int njobs,
                                                                        int s)
{
    const CombineJob &j = find_job(jobs, njobs, blockIdx.x);
    combine_direct_body<false, false, kMaxKS>(blockIdx.x - j.block0, j.n, s, j.m, j.X, j.ldx, nullptr, 0, j.C, j.ldc,
                                              static_cast<double *>(j.T), j.ldt, nullptr, 0, j.fields_per_wg, j.ntiles,
                                              NoiseArgs{BKO_NOISE_NONE, 0.0, 0, 0});
}

// Grid of the combination kernels: 64-cell tiles, the fields split so that
// the grid has a few thousand workgroups.
inline void combine_grid(int64_t n, int64_t m, uint32_t &ntiles, int64_t &fields_per_wg, uint64_t &nb)
{
    ntiles = static_cast<uint32_t>((n + kTM - 1) / kTM);
    const int64_t ftiles = (m + kTN - 1) / kTN;
    int64_t splits = std::max<int64_t>(1, std::min<int64_t>(ftiles, (8192 + ntiles - 1) / ntiles));
    fields_per_wg = ((ftiles + splits - 1) / splits) * kTN;
    splits = (m + fields_per_wg - 1) / fields_per_wg;
    nb = static_cast<uint64_t>(ntiles) * splits;
}

bko_status run_direct(int64_t n, int s, int64_t m, const double *X, int64_t ldx, const double *Y, int64_t ldy,
                      const double *C, int64_t ldc, double *T, int64_t ldt, double *F, int64_t ldf, hipStream_t stream,
                      NoiseArgs na = NoiseArgs{BKO_NOISE_NONE, 0.0, 0, 0})
{
    uint32_t ntiles;
    int64_t fields_per_wg;
    uint64_t nb;
    combine_grid(n, m, ntiles, fields_per_wg, nb);
    if (nb > 0x7fffffffu) {
        set_error("combine grid too large");
        return BKO_EINVAL;
    }
    const dim3 grid(static_cast<uint32_t>(nb)), block(kThreads);
#define BKO_DIRECT(D, E, KS)                                                                                           \
    hipLaunchKernelGGL((combine_direct_kernel<D, E, KS>), grid, block, 0, stream, n, s, m, X, ldx, Y, ldy, C, ldc, T, \
                       ldt, F, ldf, fields_per_wg, ntiles, na)
    // the noise epilogue (Philox state) is compiled only into the noisy
    // variant, so that the others keep their registers for occupancy
    const int ks = (s + 3) / 4;
    const bool noisy = na.kind != BKO_NOISE_NONE;
    if (Y && noisy) {
        set_error("the one-pass combination takes no noise term");
        return BKO_EINVAL;
    }
    if (Y) {
        if (ks <= 4) BKO_DIRECT(true, false, 4);
        else if (ks <= 8) BKO_DIRECT(true, false, 8);
        else BKO_DIRECT(true, false, 16);
    } else if (noisy) {
        if (ks <= 4) BKO_DIRECT(false, true, 4);
        else if (ks <= 8) BKO_DIRECT(false, true, 8);
        else BKO_DIRECT(false, true, 16);
    } else {
        if (ks <= 4) BKO_DIRECT(false, false, 4);
        else if (ks <= 8) BKO_DIRECT(false, false, 8);
        else BKO_DIRECT(false, false, 16);
    }
#undef BKO_DIRECT
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class Tx, class Tc, class Tt>
bko_status run_wide(int64_t n, int s, int64_t m, const void *X, int64_t ldx, const void *C, int64_t ldc, void *T,
                    int64_t ldt, hipStream_t stream)
{
    const uint32_t ntiles = static_cast<uint32_t>((n + kWideTM - 1) / kWideTM);
    const int64_t fblocks = (m + kWideF - 1) / kWideF;
    // split the fields so that the grid has a few thousand workgroups
    int64_t splits = std::max<int64_t>(1, std::min<int64_t>(fblocks, (2048 + ntiles - 1) / ntiles));
    const int64_t fields_per_wg = ((fblocks + splits - 1) / splits) * kWideF;
    splits = (m + fields_per_wg - 1) / fields_per_wg;
    const uint64_t nb = static_cast<uint64_t>(ntiles) * splits;
    if (nb > 0x7fffffffu) {
        set_error("combine grid too large");
        return BKO_EINVAL;
    }
    const int vec_ok = (reinterpret_cast<uintptr_t>(T) % 16 == 0) && ((ldt * sizeof(Tt)) % 16 == 0);
    hipLaunchKernelGGL((combine_wide_kernel<Tx, Tc, Tt>), dim3(static_cast<uint32_t>(nb)), dim3(kWideThreads), 0,
                       stream, n, s, m, static_cast<const Tx *>(X), ldx, static_cast<const Tc *>(C), ldc,
                       static_cast<Tt *>(T), ldt, fields_per_wg, ntiles, vec_ok);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <int kMode, class Tx, class Tc, class Tt>
bko_status run(int64_t n, int s, int64_t m, const void *X, int64_t ldx, const void *C, int64_t ldc, void *T,
               int64_t ldt, hipStream_t stream)
{
    if constexpr (kMode == kBF16 && !std::is_same<Tt, double>::value)
        return run_wide<Tx, Tc, Tt>(n, s, m, X, ldx, C, ldc, T, ldt, stream);
    using TR = ModeTraits<kMode>;
    const uint32_t ntiles = static_cast<uint32_t>((n + kTM - 1) / kTM);
    const int64_t ftiles = (m + kTN - 1) / kTN;
    // split the fields so that the grid has a few thousand workgroups
    int64_t splits = std::max<int64_t>(1, std::min<int64_t>(ftiles, (8192 + ntiles - 1) / ntiles));
    const int64_t fields_per_wg = ((ftiles + splits - 1) / splits) * kTN;
    splits = (m + fields_per_wg - 1) / fields_per_wg;
    const uint64_t nb = static_cast<uint64_t>(ntiles) * splits;
    if (nb > 0x7fffffffu) {
        set_error("combine grid too large");
        return BKO_EINVAL;
    }
    const int ksteps = (s + TR::kK - 1) / TR::kK;
    const int s_pad = ksteps * TR::kK;
    const int cstride = kMode == kBF16 ? s_pad + 8 : s_pad + 1;
    const int ostride = kTM + (sizeof(typename TR::Acc) == 8 ? 2 : 4);
    const size_t cbytes = sizeof(typename TR::Stage) * kTN * cstride;
    const size_t smem = std::max(cbytes, sizeof(typename TR::Acc) * kTN * ostride);
    const int vec_ok = (reinterpret_cast<uintptr_t>(T) % 16 == 0) && ((ldt * sizeof(Tt)) % 16 == 0);
    hipLaunchKernelGGL((combine_kernel<kMode, Tx, Tc, Tt>), dim3(static_cast<uint32_t>(nb)), dim3(kThreads), smem,
                       stream, n, s, m, static_cast<const Tx *>(X), ldx, static_cast<const Tc *>(C), ldc,
                       static_cast<Tt *>(T), ldt, fields_per_wg, ntiles, vec_ok);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <int kMode, class Tx, class Tc>
bko_status by_out(int64_t n, int s, int64_t m, const void *X, int64_t ldx, const void *C, int64_t ldc, void *T,
                  int64_t ldt, bko_dtype t_t, hipStream_t stream)
{
    switch (t_t) {
    case BKO_F64: return run<kMode, Tx, Tc, double>(n, s, m, X, ldx, C, ldc, T, ldt, stream);
    case BKO_F32: return run<kMode, Tx, Tc, float>(n, s, m, X, ldx, C, ldc, T, ldt, stream);
    default: return run<kMode, Tx, Tc, bf16>(n, s, m, X, ldx, C, ldc, T, ldt, stream);
    }
}

template <int kMode, class Tx>
bko_status by_c(int64_t n, int s, int64_t m, const void *X, int64_t ldx, const void *C, int64_t ldc, bko_dtype c_t,
                void *T, int64_t ldt, bko_dtype t_t, hipStream_t stream)
{
    switch (c_t) {
    case BKO_F64: return by_out<kMode, Tx, double>(n, s, m, X, ldx, C, ldc, T, ldt, t_t, stream);
    case BKO_F32: return by_out<kMode, Tx, float>(n, s, m, X, ldx, C, ldc, T, ldt, t_t, stream);
    default: return by_out<kMode, Tx, bf16>(n, s, m, X, ldx, C, ldc, T, ldt, t_t, stream);
    }
}

template <int kMode>
bko_status by_x(int64_t n, int s, int64_t m, const void *X, int64_t ldx, bko_dtype x_t, const void *C, int64_t ldc,
                bko_dtype c_t, void *T, int64_t ldt, bko_dtype t_t, hipStream_t stream)
{
    switch (x_t) {
    case BKO_F64: return by_c<kMode, double>(n, s, m, X, ldx, C, ldc, c_t, T, ldt, t_t, stream);
    case BKO_F32: return by_c<kMode, float>(n, s, m, X, ldx, C, ldc, c_t, T, ldt, t_t, stream);
    default: return by_c<kMode, bf16>(n, s, m, X, ldx, C, ldc, c_t, T, ldt, t_t, stream);
    }
}

template <int kMode, class Tt>
bko_status run_group(const std::vector<CombineJob> &jobs, uint32_t total, int s, const void *jobs_dev,
                     hipStream_t stream)
{
    using TR = ModeTraits<kMode>;
    const int ksteps = (s + TR::kK - 1) / TR::kK;
    const int s_pad = ksteps * TR::kK;
    const int cstride = kMode == kBF16 ? s_pad + 8 : s_pad + 1;
    const int ostride = kTM + (sizeof(typename TR::Acc) == 8 ? 2 : 4);
    const size_t smem = std::max(sizeof(typename TR::Stage) * kTN * cstride, sizeof(typename TR::Acc) * kTN * ostride);
    hipLaunchKernelGGL((combine_group_kernel<kMode, Tt>), dim3(total), dim3(kThreads), smem, stream,
                       static_cast<const CombineJob *>(jobs_dev), static_cast<int>(jobs.size()), s);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <int kMode>
bko_status group_by_out(const std::vector<CombineJob> &jobs, uint32_t total, int s, const void *jobs_dev,
                        bko_dtype t_t, hipStream_t stream)
{
    switch (t_t) {
    case BKO_F64: return run_group<kMode, double>(jobs, total, s, jobs_dev, stream);
    case BKO_F32: return run_group<kMode, float>(jobs, total, s, jobs_dev, stream);
    default: return run_group<kMode, bf16>(jobs, total, s, jobs_dev, stream);
    }
}

}  // namespace

bko_status launch_combine(int64_t n, int s, int64_t m, const void *X, int64_t ldx, bko_dtype x_t, const void *C,
                          int64_t ldc, bko_dtype c_t, void *T, int64_t ldt, bko_dtype t_t, bko_dtype compute,
                          hipStream_t stream)
{
    if (compute == BKO_F64 && x_t == BKO_F64 && c_t == BKO_F64 && t_t == BKO_F64)
        return run_direct(n, s, m, static_cast<const double *>(X), ldx, nullptr, 0, static_cast<const double *>(C), ldc,
                          static_cast<double *>(T), ldt, nullptr, 0, stream);
    switch (compute) {
    case BKO_F64: return by_x<kF64>(n, s, m, X, ldx, x_t, C, ldc, c_t, T, ldt, t_t, stream);
    case BKO_F32: return by_x<kF32>(n, s, m, X, ldx, x_t, C, ldc, c_t, T, ldt, t_t, stream);
    default: return by_x<kBF16>(n, s, m, X, ldx, x_t, C, ldc, c_t, T, ldt, t_t, stream);
    }
}

bko_status launch_combine_dual(int64_t n, int s, int64_t m, const double *X, int64_t ldx, const double *Y, int64_t ldy,
                               const double *C, int64_t ldc, double *T, int64_t ldt, double *F, int64_t ldf,
                               hipStream_t stream)
{
    return run_direct(n, s, m, X, ldx, Y, ldy, C, ldc, T, ldt, F, ldf, stream);
}

bko_status launch_combine_noisy(int64_t n, int s, int64_t m, const double *X, int64_t ldx, const double *C, int64_t ldc,
                                double *T, int64_t ldt, int kind, double amp, uint64_t seed, uint64_t field_offset,
                                hipStream_t stream)
{
    return run_direct(n, s, m, X, ldx, nullptr, 0, C, ldc, T, ldt, nullptr, 0, stream,
                      NoiseArgs{kind, amp, seed, field_offset});
}

bko_status launch_noise_fill(int64_t n, int64_t m, double *E, int64_t lde, int kind, double amp, uint64_t seed,
                             uint64_t field_offset, hipStream_t stream)
{
    if (n == 0 || m == 0) return BKO_OK;
    const unsigned bx = static_cast<unsigned>(std::min<int64_t>((n + kThreads - 1) / kThreads, 1024));
    hipLaunchKernelGGL(noise_fill_kernel, dim3(bx, static_cast<unsigned>(m)), dim3(kThreads), 0, stream, n, m, E, lde,
                       NoiseArgs{kind, amp, seed, field_offset});
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status launch_normalize_weights(int s, int64_t m, double *C, int64_t ldc, double min_abs, int *flags,
                                    hipStream_t stream)
{
    if (m == 0) return BKO_OK;
    hipLaunchKernelGGL(normalize_weights_kernel, dim3(static_cast<unsigned>((m + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, stream, s, m, C, ldc, min_abs, flags);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

size_t combine_group_job_bytes(int nchips) { return sizeof(CombineJob) * static_cast<size_t>(nchips); }

bko_status launch_combine_group(int nchips, const int64_t *n, int s, const int *m, const double *const *X,
                                const int64_t *ldx, const double *const *C, const int64_t *ldc, void *const *T,
                                const int64_t *ldt, bko_dtype t_t, bko_dtype compute, int64_t fields_per_wg,
                                void *jobs_dev, std::vector<unsigned char> &host_jobs, hipStream_t stream)
{
    int64_t mmax = 0, tiles = 0;
    for (int c = 0; c < nchips; ++c) {
        mmax = std::max<int64_t>(mmax, m[c]);
        if (m[c] > 0) tiles += (n[c] + kTM - 1) / kTM;
    }
    if (mmax == 0) return BKO_OK;
    // fields per workgroup: all of a chip's fields in one workgroup per
    // tile, halved (in whole 64-field steps) until the grid has a few
    // thousand workgroups; fields_per_wg > 0 fixes it
    int64_t fpw = fields_per_wg;
    if (fpw <= 0) {
        fpw = (mmax + kTN - 1) / kTN * kTN;
        while (fpw > kTN) {
            int64_t total = 0;
            for (int c = 0; c < nchips; ++c)
                if (m[c] > 0) total += ((n[c] + kTM - 1) / kTM) * ((m[c] + fpw - 1) / fpw);
            if (total >= 8192) break;
            fpw = std::max<int64_t>(kTN, (fpw / 2 + kTN - 1) / kTN * kTN);
        }
    }
    std::vector<CombineJob> jobs;
    uint64_t total = 0;
    for (int c = 0; c < nchips; ++c) {
        if (m[c] <= 0) continue;
        CombineJob j{};
        j.X = X[c];
        j.C = C[c];
        j.T = T[c];
        j.ldx = ldx[c];
        j.ldc = ldc[c];
        j.ldt = ldt[c];
        j.n = n[c];
        j.m = m[c];
        j.fields_per_wg = fpw;
        j.ntiles = static_cast<uint32_t>((n[c] + kTM - 1) / kTM);
        j.block0 = static_cast<uint32_t>(total);
        j.vec_ok = (reinterpret_cast<uintptr_t>(T[c]) % 16 == 0) && ((ldt[c] * dtype_size(t_t)) % 16 == 0);
        total += static_cast<uint64_t>(j.ntiles) * ((m[c] + fpw - 1) / fpw);
        jobs.push_back(j);
    }
    if (total > 0x7fffffffu) {
        set_error("grouped combination of %llu workgroups too large", (unsigned long long)total);
        return BKO_EINVAL;
    }
    const size_t bytes = sizeof(CombineJob) * jobs.size();
    host_jobs.resize(bytes);
    std::memcpy(host_jobs.data(), jobs.data(), bytes);
    BKO_HIP(hipMemcpyAsync(jobs_dev, host_jobs.data(), bytes, hipMemcpyHostToDevice, stream));
    const uint32_t tot = static_cast<uint32_t>(total);
    const auto *jd = static_cast<const CombineJob *>(jobs_dev);
    const int njobs = static_cast<int>(jobs.size());
    if (compute == BKO_F64 && t_t == BKO_F64) {
        const int ks = (s + 3) / 4;
        if (ks <= 4) hipLaunchKernelGGL((combine_direct_group_kernel<4>), dim3(tot), dim3(kThreads), 0, stream, jd, njobs, s);
        else if (ks <= 8) hipLaunchKernelGGL((combine_direct_group_kernel<8>), dim3(tot), dim3(kThreads), 0, stream, jd, njobs, s);
        else hipLaunchKernelGGL((combine_direct_group_kernel<16>), dim3(tot), dim3(kThreads), 0, stream, jd, njobs, s);
        BKO_HIP(hipGetLastError());
        return BKO_OK;
    }
    switch (compute) {
    case BKO_F64: return group_by_out<kF64>(jobs, tot, s, jobs_dev, t_t, stream);
    case BKO_F32: return group_by_out<kF32>(jobs, tot, s, jobs_dev, t_t, stream);
    default: return group_by_out<kBF16>(jobs, tot, s, jobs_dev, t_t, stream);
    }
}

}  // namespace bko
