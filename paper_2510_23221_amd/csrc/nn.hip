// Learned initial guess for the block solve: a 4-level convolutional
// encoder-decoder trained and run with the kernels of this file.  The
// network is the project's addition (it supplies X0 of the block solve of
// Sec. III-A; the paper has no learned component on this path).
//
// Tensors are FP32, layout (N, C, H, W).  Filters are kept as FP32 master
// parameters (updated by Adam) and a BF16 copy that every convolution reads
// (BF16 weights, FP32 accumulation).  Flat parameter order: for each layer
// of the table below, its filter (Cout, Cin, K, K) row-major, then its bias
// (Cout).
//
// Layers (3 x 3 "same" convolutions with bias and ReLU unless noted):
//   0,1   Cin -> w1 -> w1           at H            (skip s1 = output of 1)
//   2,3   pool(s1): w1 -> w2 -> w2  at H/2          (skip s2)
//   4,5   pool(s2): w2 -> w3 -> w3  at H/4          (skip s3)
//   6,7   pool(s3): w3 -> w4 -> w4  at H/8
//   8,9   [up(7), s3]: w4+w3 -> w3 -> w3   at H/4
//   10,11 [up(9), s2]: w3+w2 -> w2 -> w2   at H/2
//   12,13 [up(11), s1]: w2+w1 -> w1 -> w1  at H
//   14    1 x 1, w1 -> Cout, no ReLU
// with w1 = base, w2 = 2 base, w3 = w4 = 4 base.  pool is 2 x 2 averaging,
// up is nearest 2x upsampling, [a, b] concatenation along channels.
//
// The convolution reads its input through a mode so that pooling and the
// upsample-and-concatenate of the decoder never materialise: mode 0 reads A;
// mode 1 reads the 2 x 2 average of A (A at twice the resolution); mode 2
// reads channel c < Ca of A at half resolution and channel c >= Ca of B.
// The same kernel computes the input gradient (flipped, transposed filters);
// a second kernel forms the filter and bias gradients as per-split partials
// summed in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.hpp"

namespace bko {

namespace {

constexpr int kNT = 256;   // threads per workgroup
constexpr int kTH = 16;    // output tile rows (forward)
constexpr int kTW = 32;    // output tile columns (forward)
constexpr int kCO = 32;    // output channels per workgroup
constexpr int kCI = 8;     // input channels per LDS stage
constexpr int kGH = 8;     // pixel tile rows of the filter gradient

__device__ inline float bf16f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

__device__ inline uint16_t f2bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

// The convolution input seen through its mode (zero outside the image).
struct ConvIn {
    const float *A;
    const float *B;
    int Ca, Cb;  // channels of A and B (Cb = 0 unless mode 2)
    int mode;
};

__device__ inline float read_in(const ConvIn &in, int n, int c, int y, int x, int H, int W)
{
    if (y < 0 || y >= H || x < 0 || x >= W) return 0.0f;
    if (in.mode == 0) return in.A[((static_cast<int64_t>(n) * in.Ca + c) * H + y) * W + x];
    if (in.mode == 1) {
        const int H2 = 2 * H, W2 = 2 * W;
        const float *p = in.A + ((static_cast<int64_t>(n) * in.Ca + c) * H2 + 2 * y) * W2 + 2 * x;
        return 0.25f * ((p[0] + p[1]) + (p[W2] + p[W2 + 1]));
    }
    if (c < in.Ca) {
        const int Hh = H / 2, Wh = W / 2;
        return in.A[((static_cast<int64_t>(n) * in.Ca + c) * Hh + (y >> 1)) * Wh + (x >> 1)];
    }
    return in.B[((static_cast<int64_t>(n) * in.Cb + (c - in.Ca)) * H + y) * W + x];
}

// out[n, o, y, x] = bias[o] + sum_{i, p, q} w(o, i, p, q) in[n, i, y + p - r, x + q - r]
// (ReLU if relu).  w(o, i, p, q) = wgt[o][i][p][q], or with transposed != 0
// wgt[i][o][K-1-p][K-1-q] (the input gradient of a layer with Ci and Co
// swapped).  Grid: (W tiles, H tiles, N * output-channel tiles).  Thread t
// owns two horizontally adjacent pixels and kCO output channels.
template <int K>
__global__ __launch_bounds__(kNT) void conv_kernel(ConvIn in, int N, int H, int W, int Ci, int Co,
                                                   const uint16_t *__restrict__ wgt, int transposed,
                                                   const float *__restrict__ bias, float *__restrict__ out, int relu)
{
    constexpr int R = K / 2;
    constexpr int IH = kTH + 2 * R, IW = kTW + 2 * R;
    constexpr int KK = K * K;
    constexpr int KP = (KK + 3) / 4 * 4;  // padded taps (float4 reads)
    __shared__ float sIn[kCI][IH][IW + 1];
    __shared__ __align__(16) float sW[kCI][kCO][KP];
    const int tid = threadIdx.x;
    const int coTiles = (Co + kCO - 1) / kCO;
    const int n = blockIdx.z / coTiles, co0 = (blockIdx.z % coTiles) * kCO;
    const int y0 = blockIdx.y * kTH, x0 = blockIdx.x * kTW;
    const int ty = tid / (kTW / 2), tx = (tid % (kTW / 2)) * 2;
    float acc[kCO][2];
#pragma unroll
    for (int o = 0; o < kCO; ++o) acc[o][0] = acc[o][1] = 0.0f;

    for (int ci0 = 0; ci0 < Ci; ci0 += kCI) {
        for (int e = tid; e < kCI * IH * IW; e += kNT) {
            const int c = e / (IH * IW), r = (e / IW) % IH, q = e % IW;
            sIn[c][r][q] = ci0 + c < Ci ? read_in(in, n, ci0 + c, y0 + r - R, x0 + q - R, H, W) : 0.0f;
        }
        for (int e = tid; e < kCI * kCO * KK; e += kNT) {
            const int c = e / (kCO * KK), o = (e / KK) % kCO, t = e % KK;
            const int i = ci0 + c, oo = co0 + o;
            float v = 0.0f;
            if (i < Ci && oo < Co) {
                const int p = t / K, q = t % K;
                const int64_t idx = transposed
                                        ? ((static_cast<int64_t>(i) * Co + oo) * K + (K - 1 - p)) * K + (K - 1 - q)
                                        : ((static_cast<int64_t>(oo) * Ci + i) * K + p) * K + q;
                v = bf16f(wgt[idx]);
            }
            sW[c][o][t] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int c = 0; c < kCI; ++c) {
            float win[K][K + 1];
#pragma unroll
            for (int p = 0; p < K; ++p)
#pragma unroll
                for (int q = 0; q < K + 1; ++q) win[p][q] = sIn[c][ty + p][tx + q];
#pragma unroll
            for (int o = 0; o < kCO; ++o) {
                float w[KP];
#pragma unroll
                for (int t = 0; t < KP; t += 4) *reinterpret_cast<float4 *>(&w[t]) = *reinterpret_cast<const float4 *>(&sW[c][o][t]);
#pragma unroll
                for (int p = 0; p < K; ++p)
#pragma unroll
                    for (int q = 0; q < K; ++q) {
                        acc[o][0] = fmaf(w[p * K + q], win[p][q], acc[o][0]);
                        acc[o][1] = fmaf(w[p * K + q], win[p][q + 1], acc[o][1]);
                    }
            }
        }
        __syncthreads();
    }
    const int y = y0 + ty;
    if (y >= H) return;
#pragma unroll
    for (int o = 0; o < kCO; ++o) {
        const int oo = co0 + o;
        if (oo >= Co) break;
        const float b = bias ? bias[oo] : 0.0f;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int x = x0 + tx + d;
            if (x < W) {
                float v = acc[o][d] + b;
                if (relu) v = fmaxf(v, 0.0f);
                out[((static_cast<int64_t>(n) * Co + oo) * H + y) * W + x] = v;
            }
        }
    }
}

// The forward convolution on the BF16 matrix cores, for inference: the
// same output tiles as conv_kernel (kTH x kTW pixels x kCO output channels
// per workgroup), as an implicit GEMM over k = (tap, input channel).  Each
// stage brings kMCI input channels into LDS channel-last in BF16 (inputs
// rounded to nearest even, the weights are BF16 already), so that a lane's
// eight k values of one 32-deep matrix-core step (one tap, eight
// consecutive channels) are one 16-byte LDS read; taps are padded to an even
// count with zero weights.  Wave w owns tile rows 4w .. 4w + 3 (eight
// 16-pixel blocks) and both 16-channel blocks; FP32 accumulation, bias and
// ReLU in the epilogue.
constexpr int kMCI = 16;  // input channels per LDS stage of the matrix-core convolution

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef __bf16 mbf8 __attribute__((ext_vector_type(8)));

template <int K>
__global__ __launch_bounds__(kNT) void conv_mfma_kernel(ConvIn in, int N, int H, int W, int Ci, int Co,
                                                        const uint16_t *__restrict__ wgt,
                                                        const float *__restrict__ bias, float *__restrict__ out,
                                                        int relu)
{
    constexpr int R = K / 2;
    constexpr int IH = kTH + 2 * R, IW = kTW + 2 * R;
    constexpr int KK = K * K;
    constexpr int TP = (KK + 1) / 2 * 2;  // taps padded to pairs: a 32-deep step is two taps x 16 channels
    static_assert(kTH == 16 && kTW == 32 && kCO == 32 && kNT == 256, "tile mapping of the matrix-core convolution");
    __shared__ __align__(16) uint16_t sIn[IH * IW * kMCI];  // [row][col][channel]
    __shared__ __align__(16) uint16_t sW[kCO * TP * kMCI];  // [out channel][tap][channel]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int coTiles = (Co + kCO - 1) / kCO;
    const int n = blockIdx.z / coTiles, co0 = (blockIdx.z % coTiles) * kCO;
    const int y0 = blockIdx.y * kTH, x0 = blockIdx.x * kTW;
    mf4 acc[8][2];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) acc[b][ob] = mf4{0.f, 0.f, 0.f, 0.f};

    for (int ci0 = 0; ci0 < Ci; ci0 += kMCI) {
        // a thread takes eight channels of one pixel (each read coalesced
        // across the threads of a row) and writes them as one 16-byte vector
        for (int e = tid; e < 2 * IH * IW; e += kNT) {
            const int g = e / (IH * IW), r = (e / IW) % IH, q = e % IW;
            uint32_t pk[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int c0 = ci0 + 8 * g + 2 * h;
                const float v0 = c0 < Ci ? read_in(in, n, c0, y0 + r - R, x0 + q - R, H, W) : 0.0f;
                const float v1 = c0 + 1 < Ci ? read_in(in, n, c0 + 1, y0 + r - R, x0 + q - R, H, W) : 0.0f;
                pk[h] = static_cast<uint32_t>(f2bf16(v0)) | (static_cast<uint32_t>(f2bf16(v1)) << 16);
            }
            *reinterpret_cast<uint4 *>(&sIn[(r * IW + q) * kMCI + 8 * g]) = uint4{pk[0], pk[1], pk[2], pk[3]};
        }
        for (int e = tid; e < kCO * TP * kMCI; e += kNT) {
            const int o = e / (TP * kMCI), t = (e / kMCI) % TP, c = e % kMCI;
            const int oo = co0 + o, i = ci0 + c;
            sW[e] = (oo < Co && i < Ci && t < KK) ? wgt[(static_cast<int64_t>(oo) * Ci + i) * KK + t] : uint16_t(0);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < TP / 2; ++j) {
            const int t = 2 * j + (lg >> 1);  // this lane group's tap and channels
            const int cb = 8 * (lg & 1);
            const int p = t < KK ? t / K : 0, q = t < KK ? t % K : 0;  // a padding tap reads in bounds (zero weight)
            mbf8 b[2];
#pragma unroll
            for (int ob = 0; ob < 2; ++ob)
                b[ob] = *reinterpret_cast<const mbf8 *>(&sW[((ob * 16 + li) * TP + t) * kMCI + cb]);
#pragma unroll
            for (int pb = 0; pb < 8; ++pb) {
                const int row = 4 * wave + (pb >> 1), col = 16 * (pb & 1) + li;
                const mbf8 a = *reinterpret_cast<const mbf8 *>(&sIn[((row + p) * IW + col + q) * kMCI + cb]);
#pragma unroll
                for (int ob = 0; ob < 2; ++ob) acc[pb][ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[ob], acc[pb][ob], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // result register r of lane (li, lg): pixel 4 lg + r of the block, output channel li of the channel block
#pragma unroll
    for (int pb = 0; pb < 8; ++pb) {
        const int y = y0 + 4 * wave + (pb >> 1);
        if (y >= H) continue;
#pragma unroll
        for (int ob = 0; ob < 2; ++ob) {
            const int oo = co0 + ob * 16 + li;
            if (oo >= Co) continue;
            const float bv = bias ? bias[oo] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = x0 + 16 * (pb & 1) + 4 * lg + r;
                if (x < W) {
                    float v = acc[pb][ob][r] + bv;
                    if (relu) v = fmaxf(v, 0.0f);
                    out[((static_cast<int64_t>(n) * Co + oo) * H + y) * W + x] = v;
                }
            }
        }
    }
}

// Filter and bias gradient partials of one split:
//   part[split][o][i][p][q] = sum over the split's pixels of g[n,o,y,x] in[n,i,y+p-r,x+q-r]
//   bpart[split][o]         = sum over the split's pixels of g[n,o,y,x]
// Grid: (output-channel tiles * input-channel tiles, splits).  Thread t owns
// (o, i) = (t / kCI, t % kCI) of the tile and its K*K taps; pixel tiles of
// kGH x kTW are walked split, split + splits, ...
template <int K>
__global__ __launch_bounds__(kNT) void wgrad_kernel(ConvIn in, const float *__restrict__ g, int N, int H, int W, int Ci,
                                                    int Co, int splits, float *__restrict__ part,
                                                    float *__restrict__ bpart)
{
    constexpr int R = K / 2;
    constexpr int IH = kGH + 2 * R, IW = kTW + 2 * R;
    constexpr int KK = K * K;
    __shared__ float sG[kCO][kGH * (kTW + 1) + 1];
    __shared__ float sIn[kCI][IH][IW + 2];
    const int tid = threadIdx.x;
    const int ciTiles = (Ci + kCI - 1) / kCI;
    const int co0 = (blockIdx.x / ciTiles) * kCO, ci0 = (blockIdx.x % ciTiles) * kCI;
    const int split = blockIdx.y;
    const int ol = tid / kCI, il = tid % kCI;
    const int tilesX = (W + kTW - 1) / kTW, tilesY = (H + kGH - 1) / kGH;
    const int ntiles = N * tilesY * tilesX;
    float acc[KK];
#pragma unroll
    for (int t = 0; t < KK; ++t) acc[t] = 0.0f;
    float bacc = 0.0f;
    for (int pt = split; pt < ntiles; pt += splits) {
        const int n = pt / (tilesY * tilesX);
        const int y0 = ((pt / tilesX) % tilesY) * kGH, x0 = (pt % tilesX) * kTW;
        for (int e = tid; e < kCO * kGH * kTW; e += kNT) {
            const int o = e / (kGH * kTW), r = (e / kTW) % kGH, q = e % kTW;
            const int y = y0 + r, x = x0 + q, oo = co0 + o;
            sG[o][r * (kTW + 1) + q] =
                (oo < Co && y < H && x < W) ? g[((static_cast<int64_t>(n) * Co + oo) * H + y) * W + x] : 0.0f;
        }
        for (int e = tid; e < kCI * IH * IW; e += kNT) {
            const int c = e / (IH * IW), r = (e / IW) % IH, q = e % IW;
            sIn[c][r][q] = ci0 + c < Ci ? read_in(in, n, ci0 + c, y0 + r - R, x0 + q - R, H, W) : 0.0f;
        }
        __syncthreads();
        for (int r = 0; r < kGH; ++r) {
            // sliding K x K window along the row
            float win[K][K];
#pragma unroll
            for (int p = 0; p < K; ++p)
#pragma unroll
                for (int q = 0; q < K - 1; ++q) win[p][q + 1] = sIn[il][r + p][q];
            for (int x = 0; x < kTW; ++x) {
#pragma unroll
                for (int p = 0; p < K; ++p) {
#pragma unroll
                    for (int q = 0; q < K - 1; ++q) win[p][q] = win[p][q + 1];
                    win[p][K - 1] = sIn[il][r + p][x + K - 1];
                }
                const float gv = sG[ol][r * (kTW + 1) + x];
#pragma unroll
                for (int p = 0; p < K; ++p)
#pragma unroll
                    for (int q = 0; q < K; ++q) acc[p * K + q] = fmaf(gv, win[p][q], acc[p * K + q]);
                bacc += gv;
            }
        }
        __syncthreads();
    }
    const int oo = co0 + ol, ii = ci0 + il;
    if (oo < Co && ii < Ci) {
        float *dst = part + ((static_cast<int64_t>(split) * Co + oo) * Ci + ii) * KK;
#pragma unroll
        for (int t = 0; t < KK; ++t) dst[t] = acc[t];
    }
    if (ci0 == 0 && il == 0 && oo < Co) bpart[static_cast<int64_t>(split) * Co + oo] = bacc;
}

// gw = sum over splits of the partials (in split order); gb likewise.
__global__ __launch_bounds__(kNT) void wgrad_reduce_kernel(const float *__restrict__ part,
                                                           const float *__restrict__ bpart, int splits, int64_t nw,
                                                           int Co, float *__restrict__ gw, float *__restrict__ gb)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e < nw) {
        float t = 0.0f;
        for (int s = 0; s < splits; ++s) t += part[static_cast<int64_t>(s) * nw + e];
        gw[e] = t;
    }
    if (e < Co) {
        float t = 0.0f;
        for (int s = 0; s < splits; ++s) t += bpart[static_cast<int64_t>(s) * Co + e];
        gb[e] = t;
    }
}

// g <- g * (y > 0)
__global__ void relu_bwd_kernel(float *__restrict__ g, const float *__restrict__ y, int64_t n)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e < n && !(y[e] > 0.0f)) g[e] = 0.0f;
}

// Gradient of the pooled input (mode 1): gA[n,c,Y,X] = g[n,c,Y/2,X/2] / 4 (+ add[...]).
__global__ void pool_bwd_kernel(const float *__restrict__ g, int NC, int H, int W, const float *__restrict__ add,
                                float *__restrict__ gA)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    const int H2 = 2 * H, W2 = 2 * W;
    if (e >= static_cast<int64_t>(NC) * H2 * W2) return;
    const int X = static_cast<int>(e % W2), Y = static_cast<int>((e / W2) % H2);
    const int64_t nc = e / (static_cast<int64_t>(H2) * W2);
    float v = 0.25f * g[(nc * H + (Y >> 1)) * W + (X >> 1)];
    if (add) v += add[e];
    gA[e] = v;
}

// Split the gradient of [up(A), B] (mode 2): gA = 2 x 2 sums of channels < Ca
// at half resolution; gB = channels >= Ca.
__global__ void upcat_bwd_kernel(const float *__restrict__ g, int N, int Ca, int Cb, int H, int W,
                                 float *__restrict__ gA, float *__restrict__ gB)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    const int C = Ca + Cb;
    const int Hh = H / 2, Wh = W / 2;
    const int64_t nA = static_cast<int64_t>(N) * Ca * Hh * Wh;
    const int64_t nB = static_cast<int64_t>(N) * Cb * H * W;
    if (e < nA) {
        const int x = static_cast<int>(e % Wh), y = static_cast<int>((e / Wh) % Hh);
        const int c = static_cast<int>((e / (static_cast<int64_t>(Wh) * Hh)) % Ca);
        const int n = static_cast<int>(e / (static_cast<int64_t>(Wh) * Hh * Ca));
        const float *p = g + ((static_cast<int64_t>(n) * C + c) * H + 2 * y) * W + 2 * x;
        gA[e] = (p[0] + p[1]) + (p[W] + p[W + 1]);
    }
    if (e < nB) {
        const int64_t hw = static_cast<int64_t>(H) * W;
        const int64_t pix = e % hw;
        const int c = static_cast<int>((e / hw) % Cb);
        const int n = static_cast<int>(e / (hw * Cb));
        gB[e] = g[(static_cast<int64_t>(n) * C + Ca + c) * hw + pix];
    }
}

// d = pred - target; grad = 2 d / count; loss partial per workgroup (sum of d^2).
__global__ __launch_bounds__(kNT) void mse_kernel(const float *__restrict__ pred, const float *__restrict__ target,
                                                  int64_t n, float inv_count, float *__restrict__ grad,
                                                  float *__restrict__ lpart)
{
    __shared__ float sh[kNT];
    float s = 0.0f;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x; e < n; e += static_cast<int64_t>(gridDim.x) * kNT) {
        const float d = pred[e] - target[e];
        grad[e] = 2.0f * d * inv_count;
        s = fmaf(d, d, s);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kNT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

// Adam (Kingma and Ba, 2015) with bias correction; refreshes the BF16 copy.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ pb, int64_t n, float lr, float b1, float b2,
                            float c1, float c2, float eps)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float pi = p[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[e] = pi;
    pb[e] = f2bf16(pi);
}

__global__ void to_bf16_kernel(const float *__restrict__ p, uint16_t *__restrict__ pb, int64_t n)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e < n) pb[e] = f2bf16(p[e]);
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kNT - 1) / kNT); }

}  // namespace

// ------------------------------------------------------------------ launchers

bko_status nn_conv(const float *A, int Ca, const float *B, int Cb, int mode, int N, int H, int W, int Co, int K,
                   const uint16_t *wgt, int transposed, const float *bias, float *out, int relu, hipStream_t st)
{
    const ConvIn in{A, B, Ca, Cb, mode};
    const int Ci = Ca + Cb;
    const dim3 grid(static_cast<unsigned>((W + kTW - 1) / kTW), static_cast<unsigned>((H + kTH - 1) / kTH),
                    static_cast<unsigned>(N * ((Co + kCO - 1) / kCO)));
    if (K == 3)
        hipLaunchKernelGGL(conv_kernel<3>, grid, dim3(kNT), 0, st, in, N, H, W, Ci, Co, wgt, transposed, bias, out, relu);
    else
        hipLaunchKernelGGL(conv_kernel<1>, grid, dim3(kNT), 0, st, in, N, H, W, Ci, Co, wgt, transposed, bias, out, relu);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status nn_conv_mfma(const float *A, int Ca, const float *B, int Cb, int mode, int N, int H, int W, int Co, int K,
                        const uint16_t *wgt, const float *bias, float *out, int relu, hipStream_t st)
{
    const ConvIn in{A, B, Ca, Cb, mode};
    const int Ci = Ca + Cb;
    const dim3 grid(static_cast<unsigned>((W + kTW - 1) / kTW), static_cast<unsigned>((H + kTH - 1) / kTH),
                    static_cast<unsigned>(N * ((Co + kCO - 1) / kCO)));
    if (K == 3)
        hipLaunchKernelGGL(conv_mfma_kernel<3>, grid, dim3(kNT), 0, st, in, N, H, W, Ci, Co, wgt, bias, out, relu);
    else
        hipLaunchKernelGGL(conv_mfma_kernel<1>, grid, dim3(kNT), 0, st, in, N, H, W, Ci, Co, wgt, bias, out, relu);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

int nn_wgrad_splits(int N, int H, int W, int Ci, int Co)
{
    const int tiles = ((Co + kCO - 1) / kCO) * ((Ci + kCI - 1) / kCI);
    const int ptiles = N * ((H + kGH - 1) / kGH) * ((W + kTW - 1) / kTW);
    return std::max(1, std::min({ptiles, 64, (2048 + tiles - 1) / tiles}));
}

size_t nn_wgrad_part_floats(int N, int H, int W, int Ci, int Co, int K)
{
    const int s = nn_wgrad_splits(N, H, W, Ci, Co);
    return static_cast<size_t>(s) * (static_cast<size_t>(Co) * Ci * K * K + Co);
}

bko_status nn_wgrad(const float *A, int Ca, const float *B, int Cb, int mode, const float *g, int N, int H, int W,
                    int Co, int K, float *part, float *gw, float *gb, hipStream_t st)
{
    const ConvIn in{A, B, Ca, Cb, mode};
    const int Ci = Ca + Cb;
    const int splits = nn_wgrad_splits(N, H, W, Ci, Co);
    const int64_t nw = static_cast<int64_t>(Co) * Ci * K * K;
    float *bpart = part + static_cast<int64_t>(splits) * nw;
    const dim3 grid(static_cast<unsigned>(((Co + kCO - 1) / kCO) * ((Ci + kCI - 1) / kCI)), static_cast<unsigned>(splits));
    if (K == 3)
        hipLaunchKernelGGL(wgrad_kernel<3>, grid, dim3(kNT), 0, st, in, g, N, H, W, Ci, Co, splits, part, bpart);
    else
        hipLaunchKernelGGL(wgrad_kernel<1>, grid, dim3(kNT), 0, st, in, g, N, H, W, Ci, Co, splits, part, bpart);
    BKO_HIP(hipGetLastError());
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(blocks_for(std::max<int64_t>(nw, Co))), dim3(kNT), 0, st, part, bpart,
                       splits, nw, Co, gw, gb);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status nn_relu_bwd(float *g, const float *y, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks_for(n)), dim3(kNT), 0, st, g, y, n);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status nn_pool_bwd(const float *g, int NC, int H, int W, const float *add, float *gA, hipStream_t st)
{
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(blocks_for(static_cast<int64_t>(NC) * 4 * H * W)), dim3(kNT), 0, st, g, NC,
                       H, W, add, gA);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status nn_upcat_bwd(const float *g, int N, int Ca, int Cb, int H, int W, float *gA, float *gB, hipStream_t st)
{
    const int64_t n = std::max(static_cast<int64_t>(N) * Ca * (H / 2) * (W / 2), static_cast<int64_t>(N) * Cb * H * W);
    hipLaunchKernelGGL(upcat_bwd_kernel, dim3(blocks_for(n)), dim3(kNT), 0, st, g, N, Ca, Cb, H, W, gA, gB);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

int nn_mse_blocks(int64_t n) { return static_cast<int>(std::min<int64_t>(1024, (n + kNT - 1) / kNT)); }

bko_status nn_mse(const float *pred, const float *target, int64_t n, float *grad, float *lpart, hipStream_t st)
{
    hipLaunchKernelGGL(mse_kernel, dim3(static_cast<unsigned>(nn_mse_blocks(n))), dim3(kNT), 0, st, pred, target, n,
                       1.0f / static_cast<float>(n), grad, lpart);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status nn_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr, int t,
                   hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, static_cast<float>(t)), c2 = 1.0f - std::pow(b2, static_cast<float>(t));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(kNT), 0, st, p, g, m, v, pb, n, lr, b1, b2, c1, c2, 1e-8f);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status nn_to_bf16(const float *p, uint16_t *pb, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(kNT), 0, st, p, pb, n);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

}  // namespace bko

// ------------------------------------------------------------------ learned-start packing

namespace bko {

namespace {

// scale[j] = ||F[:, j]||_2 / sqrt(n), the RMS value (one workgroup per column, FP64)
__global__ __launch_bounds__(kNT) void colnorm64_kernel(const double *__restrict__ F, int64_t ldf, int64_t n,
                                                        double *__restrict__ scale)
{
    __shared__ double sh[kNT];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += kNT) {
        const double v = F[j * ldf + r];
        s = fma(v, v, s);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kNT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[j] = sqrt(sh[0] / static_cast<double>(n));
}

// Network input of field j: channels [0, nz) = F[:, j] / scale[j] as nz
// planes of ny x nx; [nz, 2nz) = (log k - kmu) / ksig; 2nz = hval.
__global__ void pack_kernel(int nx, int ny, int nz, const double *__restrict__ F, int64_t ldf, int m,
                            const double *__restrict__ kc, float kmu, float ksig, float hval,
                            const double *__restrict__ scale, float *__restrict__ x)
{
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int C = 2 * nz + 1;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e >= static_cast<int64_t>(m) * C * plane) return;
    const int64_t pix = e % plane;
    const int c = static_cast<int>((e / plane) % C);
    const int j = static_cast<int>(e / (plane * C));
    float v;
    if (c < nz) {
        const double s = scale[j];
        v = s > 0.0 ? static_cast<float>(F[j * ldf + c * plane + pix] / s) : 0.0f;
    } else if (c < 2 * nz) {
        v = (static_cast<float>(log(kc[(c - nz) * plane + pix])) - kmu) / ksig;
    } else {
        v = hval;
    }
    x[e] = v;
}

// Target of field j: T[:, j] / (scale[j] gain) as nz planes.
__global__ void pack_target_kernel(int64_t n, const double *__restrict__ T, int64_t ldt, int m,
                                   const double *__restrict__ scale, double gain, float *__restrict__ t)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e >= static_cast<int64_t>(m) * n) return;
    const int64_t r = e % n;
    const int j = static_cast<int>(e / n);
    const double s = scale[j] * gain;
    t[e] = s > 0.0 ? static_cast<float>(T[j * ldt + r] / s) : 0.0f;
}

// X0[:, j] = y_j * scale[j] * gain
__global__ void unpack_kernel(int64_t n, const float *__restrict__ y, int m, const double *__restrict__ scale,
                              double gain, double *__restrict__ X0, int64_t ldx)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
    if (e >= static_cast<int64_t>(m) * n) return;
    const int64_t r = e % n;
    const int j = static_cast<int>(e / n);
    X0[j * ldx + r] = static_cast<double>(y[e]) * scale[j] * gain;
}

}  // namespace

bko_status lstart_pack(int nx, int ny, int nz, const double *F, int64_t ldf, int m, const double *kc, float kmu,
                       float ksig, float hval, double *scale, float *x, hipStream_t st)
{
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    hipLaunchKernelGGL(colnorm64_kernel, dim3(static_cast<unsigned>(m)), dim3(kNT), 0, st, F, ldf, n, scale);
    BKO_HIP(hipGetLastError());
    const int64_t total = static_cast<int64_t>(m) * (2 * nz + 1) * nx * ny;
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(total)), dim3(kNT), 0, st, nx, ny, nz, F, ldf, m, kc, kmu, ksig, hval,
                       scale, x);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status lstart_pack_target(int64_t n, const double *T, int64_t ldt, int m, const double *scale, double gain,
                              float *t, hipStream_t st)
{
    hipLaunchKernelGGL(pack_target_kernel, dim3(blocks_for(static_cast<int64_t>(m) * n)), dim3(kNT), 0, st, n, T, ldt, m,
                       scale, gain, t);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status lstart_unpack(int64_t n, const float *y, int m, const double *scale, double gain, double *X0, int64_t ldx,
                         hipStream_t st)
{
    hipLaunchKernelGGL(unpack_kernel, dim3(blocks_for(static_cast<int64_t>(m) * n)), dim3(kNT), 0, st, n, y, m, scale,
                       gain, X0, ldx);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

// ------------------------------------------------------------------ the encoder-decoder

UNet::UNet(int cin_, int cout_, int base_, int H_, int W_, int batch_)
    : cin(cin_), cout(cout_), base(base_), H(H_), W(W_), batch(batch_)
{
    const int w1 = base, w2 = 2 * base, w3 = 4 * base, w4 = 4 * base;
    const int spec[15][4] = {{cin, w1, 3, 1},      {w1, w1, 3, 1},      {w1, w2, 3, 1}, {w2, w2, 3, 1},
                             {w2, w3, 3, 1},       {w3, w3, 3, 1},      {w3, w4, 3, 1}, {w4, w4, 3, 1},
                             {w4 + w3, w3, 3, 1},  {w3, w3, 3, 1},      {w3 + w2, w2, 3, 1}, {w2, w2, 3, 1},
                             {w2 + w1, w1, 3, 1},  {w1, w1, 3, 1},      {w1, cout, 1, 0}};
    const int lev[15] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
    int64_t o = 0;
    size_t f = 0;
    auto take = [&](size_t floats) {
        const size_t q = f;
        f += (floats + 63) / 64 * 64;
        return q;
    };
    size_t part = 0;
    for (int j = 0; j < 15; ++j) {
        Layer &l = L[j];
        l.ci = spec[j][0];
        l.co = spec[j][1];
        l.k = spec[j][2];
        l.relu = spec[j][3];
        l.h = H >> lev[j];
        l.w = W >> lev[j];
        l.woff = o;
        o += static_cast<int64_t>(l.co) * l.ci * l.k * l.k;
        l.boff = o;
        o += l.co;
        const size_t sz = static_cast<size_t>(batch) * l.co * l.h * l.w;
        l.act = take(sz);
        l.grad = take(sz);
        part = std::max(part, nn_wgrad_part_floats(batch, l.h, l.w, l.ci, l.co, l.k));
    }
    nparams = o;
    // gradients of the concatenated / pooled inputs (one scratch), of the skips
    size_t scratch = 0;
    for (int j : {2, 4, 6, 8, 10, 12}) scratch = std::max(scratch, static_cast<size_t>(batch) * L[j].ci * L[j].h * L[j].w);
    scratch_off = take(scratch);
    for (int q = 0; q < 3; ++q) skip_off[q] = take(static_cast<size_t>(batch) * L[2 * q + 1].co * L[2 * q + 1].h * L[2 * q + 1].w);
    part_off = take(part);
    lpart_off = take(1024);
    work_floats = f;
}

size_t UNet::state_bytes() const { return static_cast<size_t>(nparams) * (4 * sizeof(float) + sizeof(uint16_t)) + 1024; }

UNet::State UNet::state(void *p) const
{
    State s;
    float *f = static_cast<float *>(p);
    s.params = f;
    s.grads = f + nparams;
    s.m = f + 2 * nparams;
    s.v = f + 3 * nparams;
    s.pb = reinterpret_cast<uint16_t *>(f + 4 * nparams);
    return s;
}

bko_status UNet::forward(void *state_p, void *work, const float *x, int n, float *y, hipStream_t st, bool mfma) const
{
    const State S = state(state_p);
    float *w = static_cast<float *>(work);
    auto act = [&](int j) { return w + L[j].act; };
    bko_status rc;
    auto conv = [&](int j, const float *A, int Ca, const float *B, int Cb, int mode, float *out) {
        const Layer &l = L[j];
        if (mfma)
            return nn_conv_mfma(A, Ca, B, Cb, mode, n, l.h, l.w, l.co, l.k, S.pb + l.woff, S.params + l.boff, out,
                                l.relu, st);
        return nn_conv(A, Ca, B, Cb, mode, n, l.h, l.w, l.co, l.k, S.pb + l.woff, 0, S.params + l.boff, out, l.relu, st);
    };
    const int w1 = L[1].co, w2 = L[3].co, w3 = L[5].co, w4 = L[7].co;
    if ((rc = conv(0, x, cin, nullptr, 0, 0, act(0))) != BKO_OK) return rc;
    if ((rc = conv(1, act(0), w1, nullptr, 0, 0, act(1))) != BKO_OK) return rc;
    if ((rc = conv(2, act(1), w1, nullptr, 0, 1, act(2))) != BKO_OK) return rc;
    if ((rc = conv(3, act(2), w2, nullptr, 0, 0, act(3))) != BKO_OK) return rc;
    if ((rc = conv(4, act(3), w2, nullptr, 0, 1, act(4))) != BKO_OK) return rc;
    if ((rc = conv(5, act(4), w3, nullptr, 0, 0, act(5))) != BKO_OK) return rc;
    if ((rc = conv(6, act(5), w3, nullptr, 0, 1, act(6))) != BKO_OK) return rc;
    if ((rc = conv(7, act(6), w4, nullptr, 0, 0, act(7))) != BKO_OK) return rc;
    if ((rc = conv(8, act(7), w4, act(5), w3, 2, act(8))) != BKO_OK) return rc;
    if ((rc = conv(9, act(8), w3, nullptr, 0, 0, act(9))) != BKO_OK) return rc;
    if ((rc = conv(10, act(9), w3, act(3), w2, 2, act(10))) != BKO_OK) return rc;
    if ((rc = conv(11, act(10), w2, nullptr, 0, 0, act(11))) != BKO_OK) return rc;
    if ((rc = conv(12, act(11), w2, act(1), w1, 2, act(12))) != BKO_OK) return rc;
    if ((rc = conv(13, act(12), w1, nullptr, 0, 0, act(13))) != BKO_OK) return rc;
    return conv(14, act(13), w1, nullptr, 0, 0, y ? y : act(14));
}

bko_status UNet::gradient(void *state_p, void *work, const float *x, const float *target, int n, float *loss,
                          hipStream_t st) const
{
    bko_status rc;
    if ((rc = forward(state_p, work, x, n, nullptr, st)) != BKO_OK) return rc;
    const State S = state(state_p);
    float *w = static_cast<float *>(work);
    auto act = [&](int j) { return w + L[j].act; };
    auto grad = [&](int j) { return w + L[j].grad; };
    float *scratch = w + scratch_off;
    const int64_t nout = static_cast<int64_t>(n) * cout * H * W;
    if ((rc = nn_mse(act(14), target, nout, grad(14), w + lpart_off, st)) != BKO_OK) return rc;
    const int w1 = L[1].co, w2 = L[3].co, w3 = L[5].co, w4 = L[7].co;
    // layer j: ReLU mask, filter gradient from its (virtual) input, input gradient into dst
    auto back = [&](int j, const float *A, int Ca, const float *B, int Cb, int mode, float *dst) -> bko_status {
        const Layer &l = L[j];
        bko_status r;
        if (l.relu && (r = nn_relu_bwd(grad(j), act(j), static_cast<int64_t>(n) * l.co * l.h * l.w, st)) != BKO_OK) return r;
        if ((r = nn_wgrad(A, Ca, B, Cb, mode, grad(j), n, l.h, l.w, l.co, l.k, w + part_off, S.grads + l.woff,
                          S.grads + l.boff, st)) != BKO_OK)
            return r;
        if (!dst) return BKO_OK;
        // input gradient: the layer's filters flipped and transposed, at the layer's resolution
        return nn_conv(grad(j), l.co, nullptr, 0, 0, n, l.h, l.w, l.ci, l.k, S.pb + l.woff, 1, nullptr, dst, 0, st);
    };
    float *gs1 = w + skip_off[0], *gs2 = w + skip_off[1], *gs3 = w + skip_off[2];
    if ((rc = back(14, act(13), w1, nullptr, 0, 0, grad(13))) != BKO_OK) return rc;
    if ((rc = back(13, act(12), w1, nullptr, 0, 0, grad(12))) != BKO_OK) return rc;
    if ((rc = back(12, act(11), w2, act(1), w1, 2, scratch)) != BKO_OK) return rc;
    if ((rc = nn_upcat_bwd(scratch, n, w2, w1, L[12].h, L[12].w, grad(11), gs1, st)) != BKO_OK) return rc;
    if ((rc = back(11, act(10), w2, nullptr, 0, 0, grad(10))) != BKO_OK) return rc;
    if ((rc = back(10, act(9), w3, act(3), w2, 2, scratch)) != BKO_OK) return rc;
    if ((rc = nn_upcat_bwd(scratch, n, w3, w2, L[10].h, L[10].w, grad(9), gs2, st)) != BKO_OK) return rc;
    if ((rc = back(9, act(8), w3, nullptr, 0, 0, grad(8))) != BKO_OK) return rc;
    if ((rc = back(8, act(7), w4, act(5), w3, 2, scratch)) != BKO_OK) return rc;
    if ((rc = nn_upcat_bwd(scratch, n, w4, w3, L[8].h, L[8].w, grad(7), gs3, st)) != BKO_OK) return rc;
    if ((rc = back(7, act(6), w4, nullptr, 0, 0, grad(6))) != BKO_OK) return rc;
    if ((rc = back(6, act(5), w3, nullptr, 0, 1, scratch)) != BKO_OK) return rc;
    if ((rc = nn_pool_bwd(scratch, n * w3, L[6].h, L[6].w, gs3, grad(5), st)) != BKO_OK) return rc;
    if ((rc = back(5, act(4), w3, nullptr, 0, 0, grad(4))) != BKO_OK) return rc;
    if ((rc = back(4, act(3), w2, nullptr, 0, 1, scratch)) != BKO_OK) return rc;
    if ((rc = nn_pool_bwd(scratch, n * w2, L[4].h, L[4].w, gs2, grad(3), st)) != BKO_OK) return rc;
    if ((rc = back(3, act(2), w2, nullptr, 0, 0, grad(2))) != BKO_OK) return rc;
    if ((rc = back(2, act(1), w1, nullptr, 0, 1, scratch)) != BKO_OK) return rc;
    if ((rc = nn_pool_bwd(scratch, n * w1, L[2].h, L[2].w, gs1, grad(1), st)) != BKO_OK) return rc;
    if ((rc = back(1, act(0), w1, nullptr, 0, 0, grad(0))) != BKO_OK) return rc;
    if ((rc = back(0, x, cin, nullptr, 0, 0, nullptr)) != BKO_OK) return rc;
    if (loss) {
        const int nb = nn_mse_blocks(nout);
        std::vector<float> h(nb);
        BKO_HIP(hipMemcpyAsync(h.data(), w + lpart_off, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
        BKO_HIP(hipStreamSynchronize(st));
        double t = 0.0;
        for (float v : h) t += v;
        *loss = static_cast<float>(t / static_cast<double>(nout));
    }
    return BKO_OK;
}

bko_status UNet::set_params(void *state_p, const float *params, hipStream_t st)
{
    const State S = state(state_p);
    BKO_HIP(hipMemcpyAsync(S.params, params, sizeof(float) * nparams, hipMemcpyDeviceToDevice, st));
    bko_status rc;
    if ((rc = launch_zero(S.m, sizeof(float) * nparams, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(S.v, sizeof(float) * nparams, st)) != BKO_OK) return rc;
    if ((rc = launch_zero(S.grads, sizeof(float) * nparams, st)) != BKO_OK) return rc;
    step = 0;
    return nn_to_bf16(S.params, S.pb, nparams, st);
}

bko_status UNet::adam(void *state_p, float lr, hipStream_t st)
{
    const State S = state(state_p);
    ++step;
    return nn_adam(S.params, S.grads, S.m, S.v, S.pb, nparams, lr, step, st);
}

}  // namespace bko
