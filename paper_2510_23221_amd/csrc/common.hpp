// Shared device/host helpers of the gfx950 library: storage types, BF16
// conversion, launch bookkeeping and error plumbing.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/blockoa.h"

namespace bko {

// ------------------------------------------------------------------ types

// BF16 is carried as raw 16-bit words; conversions are explicit.
struct bf16 {
    uint16_t bits;
};

__device__ inline float bf16_to_f32(uint16_t b)
{
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// Round to nearest, ties to even, by gfx950's conversion instruction (one
// instruction for two values where the compiler pairs neighbouring
// conversions); NaN stays a NaN.  The empty register constraint keeps the
// FP32 value itself as the input: without it the compiler may merge a
// preceding FP64 -> FP32 conversion into one FP64 -> BF16 rounding, while
// every FP64 value the library stores as BF16 is rounded to FP32 first.
__device__ inline uint16_t f32_to_bf16(float f)
{
    asm("" : "+v"(f));
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}

template <class T> struct Conv;
template <> struct Conv<double> {
    __device__ static inline double to_f64(double v) { return v; }
    __device__ static inline float to_f32(double v) { return static_cast<float>(v); }
    __device__ static inline double from_f64(double v) { return v; }
    __device__ static inline double from_f32(float v) { return static_cast<double>(v); }
};
template <> struct Conv<float> {
    __device__ static inline double to_f64(float v) { return static_cast<double>(v); }
    __device__ static inline float to_f32(float v) { return v; }
    __device__ static inline float from_f64(double v) { return static_cast<float>(v); }
    __device__ static inline float from_f32(float v) { return v; }
};
template <> struct Conv<bf16> {
    __device__ static inline double to_f64(bf16 v) { return static_cast<double>(bf16_to_f32(v.bits)); }
    __device__ static inline float to_f32(bf16 v) { return bf16_to_f32(v.bits); }
    __device__ static inline bf16 from_f64(double v) { return bf16{f32_to_bf16(static_cast<float>(v))}; }
    __device__ static inline bf16 from_f32(float v) { return bf16{f32_to_bf16(v)}; }
};

// Accumulator-typed load / store helpers.
template <class Acc, class T> __device__ inline Acc load_as(const T *p);
template <> __device__ inline double load_as<double, double>(const double *p) { return *p; }
template <> __device__ inline double load_as<double, float>(const float *p) { return static_cast<double>(*p); }
template <> __device__ inline double load_as<double, bf16>(const bf16 *p) { return Conv<bf16>::to_f64(*p); }
template <> __device__ inline float load_as<float, double>(const double *p) { return static_cast<float>(*p); }
template <> __device__ inline float load_as<float, float>(const float *p) { return *p; }
template <> __device__ inline float load_as<float, bf16>(const bf16 *p) { return Conv<bf16>::to_f32(*p); }

template <class T, class Acc> __device__ inline T store_from(Acc v);
template <> __device__ inline double store_from<double, double>(double v) { return v; }
template <> __device__ inline float store_from<float, double>(double v) { return static_cast<float>(v); }
template <> __device__ inline bf16 store_from<bf16, double>(double v) { return Conv<bf16>::from_f64(v); }
template <> __device__ inline double store_from<double, float>(float v) { return static_cast<double>(v); }
template <> __device__ inline float store_from<float, float>(float v) { return v; }
template <> __device__ inline bf16 store_from<bf16, float>(float v) { return Conv<bf16>::from_f32(v); }

// Row of the 16x16 output block held in result register r of a lane in lane
// group g = lane / 16 (the column is lane % 16).  Measured on gfx950:
// v_mfma_f64_16x16x4f64 interleaves the rows (g + 4 r); the FP32 and BF16
// 16x16 shapes hold four consecutive rows (4 g + r).
template <bool kF64>
__device__ inline int mfma_row(int g, int r)
{
    return kF64 ? g + 4 * r : 4 * g + r;
}

inline size_t dtype_size(bko_dtype t)
{
    return t == BKO_F64 ? 8 : (t == BKO_F32 ? 4 : 2);
}

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------- XCD mapping

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  remap_block() turns the hardware order into a logical
// order in which every XCD walks a contiguous range of tiles, so stencil
// neighbours and re-read operands stay in one L2.
constexpr int kNumXcd = 8;

__device__ inline uint32_t remap_block(uint32_t bid, uint32_t nblocks)
{
    const uint32_t per = nblocks / kNumXcd;
    const uint32_t rem = nblocks % kNumXcd;
    const uint32_t xcd = bid % kNumXcd;
    const uint32_t slot = bid / kNumXcd;
    // XCDs [0, rem) own per + 1 logical blocks, the rest own per.
    const uint32_t start = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return start + slot;
}

// -------------------------------------------------------- error plumbing

void set_error(const char *fmt, ...);
bko_status hip_fail(hipError_t e, const char *what);

// LDS bytes one workgroup may allocate on the current device.
size_t device_max_lds();

// Compute units of the current device.
int device_cu_count();

#define BKO_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ::bko::hip_fail(e_, #call);        \
    } while (0)

#define BKO_CHECK(cond, ...)                                            \
    do {                                                                \
        if (!(cond)) {                                                  \
            ::bko::set_error(__VA_ARGS__);                              \
            return BKO_EINVAL;                                          \
        }                                                               \
    } while (0)

// ------------------------------------------------------------ operator

struct Operator {
    int nx, ny, nz;
    double lx, ly, lz;
    int64_t n;
    void *coeff;          // caller-owned device buffer
    // FP64 coefficient arrays (device pointers into coeff) and FP32 copies
    const double *diag64, *wx64, *wy64, *wz64;
    const float *diag32, *wx32, *wy32, *wz32;
    // the symmetrically diagonal-scaled operator S A S, S = diag(A)^(-1/2)
    // (its diagonal is 1 up to rounding), FP64 and FP32, and S in FP64
    const double *sdiag64, *swx64, *swy64, *swz64;
    const float *sdiag32, *swx32, *swy32, *swz32;
    const double *scale64;
    int precond;  // bko_precond used by the solves on this operator
    int bc[6];    // face kinds (-x, +x, -y, +y, -z, +z) and film coefficients,
    double h[6];  // for the boundary source of nonhomogeneous data
};

// Byte layout of the coefficient buffer.
struct CoeffLayout {
    size_t off[17];  // A in FP64 (4), FP32 (4); S A S in FP64 (4), FP32 (4); S in FP64
    size_t status_off;
    size_t bytes;
};
CoeffLayout coeff_layout(int64_t n);

// ------------------------------------------------------------ timing hooks

enum TimingFamily {
    kApply = 0,    // operator action over M fields
    kCombine = 1,  // T = X C
    kGram = 2,     // s x s Gram partials
    kUpdate = 3,   // block updates
    kSmall = 4,    // one-workgroup FP64 factorisations
    kSpmm = 5,     // stencil product inside the block iteration
    kResid = 6,    // FP64 residual B - A X
    kUpdateDQP = 7,  // second block update (D, Q, P)
    kNumFamilies = 8
};

// True while any timing family is selected (launches then carry events and
// are not captured into graphs).
bool timing_active();

// Events around the launches of one scope when its family is timed: by
// default two stream markers bracket the scope; launch() instead has the
// kernel's own dispatch take the two timestamps (its begin and end, as a
// kernel trace records them), so one-kernel scopes carry no marker gaps.
struct TimedLaunch {
    TimedLaunch(int family, hipStream_t s);
    ~TimedLaunch();
    template <class F, class... Args>
    void launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, Args... args)
    {
        if (ev0) {
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, static_cast<hipEvent_t>(ev0),
                                  static_cast<hipEvent_t>(ev1), 0, args...);
            in_dispatch = true;
        } else {
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
        }
    }
    int family;
    hipStream_t stream;
    void *ev0, *ev1;
    bool in_dispatch;
};

}  // namespace bko
