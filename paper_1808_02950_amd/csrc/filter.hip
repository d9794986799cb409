// Learned post-filter behind the decoder (gfx950 matrix cores: bfloat16
// operands, float32 accumulation).  Not part of the paper's method: a small
// network that removes part of the error the approximate transform leaves.
//
//   xn = (x - 128) / 64
//   a1 = relu(conv3x3(xn; W1, b1))   1 -> 32        a2 = relu(conv3x3(a1; W2, b2))   32 -> 32
//   y  = xn + conv3x3(a2; W3, b3)    32 -> 1        pixel = clip(rne(128 + 64 y), 0, 255)
// Each convolution pads its own input with zeros.  Training minimises the mean
// of (y - (orig - 128) / 64)^2 with Adam.
//
// MFMA operand layouts (v_mfma_f32_16x16x32_bf16, "mma32"; v_mfma_f32_16x16x16_bf16,
// "mma16"): lane l = 16 g + c holds row (A) / column (B) c and the K slots
// 8g..8g+7 (mma32) or 4g..4g+3 (mma16); the result lane l holds column c, rows
// 4g..4g+3.  A and B use the same slot -> k assignment, so any consistent
// placement of the contraction index is correct.
//
// Activations (32 channels, bfloat16) are stored per pixel in "slot" order:
// slot 8g + 4h + i holds channel 16h + 4g + i.  That is exactly what a lane of
// a 32-channel result holds after the two halves (h) of a product, so a result
// is written as one 16-byte store and read back as the B operand of the next
// product without moving data between lanes.
//
// Three forms:
//  * per-layer kernels (training): every layer and both input-gradient
//    convolutions, one wave per 16-column strip of 4 rows; a 32-channel input
//    row is loaded once (a step ahead) and feeds the three output rows it touches;
//  * weight-gradient kernels: pixels are the contraction index, operands are
//    transposed into LDS (channel-major) and the +-1 column shifts of the taps
//    are funnel shifts of aligned 16-byte LDS reads;
//  * the fused inference kernel: all three layers in registers, one wave per
//    strip of 14 output columns x 32 rows.  Layer 1 is evaluated at the three
//    column shifts layer 2 needs; layer 3 shifts its input one lane left and
//    right with DPP.  No activation touches memory.
#include <string.h>

#include <algorithm>
#include <cmath>

#include "adct_internal.hpp"

namespace adct {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- parameters
// flat float32, PyTorch Conv2d order
constexpr int kParams = 9857;
constexpr int kOffW1 = 0, kOffB1 = 288, kOffW2 = 320, kOffB2 = 9536, kOffW3 = 9568, kOffB3 = 9856;

// packed operands (uint16 units), each [.. ][lane 64][slots]
constexpr int kPF1 = 0;        // layer 1, mma16: [h 2][64][4], slot (g, j) = tap (row g, col j), W1 / 64
constexpr int kPF2 = 512;      // layer 2, mma32: [tap 9][h 2][64][8]
constexpr int kPF3 = 9728;     // layer 3, mma32: [dx 3][64][8], A row m < 3 = tap row dy
constexpr int kPB3 = 11264;    // input gradient of layer 3 (flipped W3^T), mma16: [h 2][64][4]
constexpr int kPB2 = 11776;    // input gradient of layer 2 (flipped W2^T), mma32: [tap 9][h 2][64][8]
constexpr int kPackHalfs = 20992;
constexpr int kPackBiasByte = kPackHalfs * 2;   // float b1[32], b2[32], b3
constexpr int64_t kPackBytes = 42496;           // rounded up to 256

__host__ __device__ constexpr int slot_channel(int s) {
    return (s & 7) < 4 ? 4 * (s >> 3) + (s & 7) : 16 + 4 * (s >> 3) + (s & 7) - 4;
}

__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_float(uint16_t b) { return __builtin_bit_cast(float, uint32_t(b) << 16); }

// two float32 -> two bfloat16 (round to nearest even), one v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// ReLU of two bfloat16 values: as signed 16-bit integers negative values are
// negative and -0 is -32768, so an integer max with 0 is the ReLU.
__device__ __forceinline__ uint32_t relu2(uint32_t v) {
    const i16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), z));
}
// keep the halves of v whose bfloat16 in m is > 0
__device__ __forceinline__ uint32_t mask2(uint32_t v, uint32_t m) {
    const uint32_t k = (int16_t(m & 0xffffu) > 0 ? 0xffffu : 0u) | (int16_t(m >> 16) > 0 ? 0xffff0000u : 0u);
    return v & k;
}

__device__ __forceinline__ f32x4 mma32(const uint4 a, const uint4 b, const f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma16(const uint2 a, const uint2 b, const f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(i16x4, a), __builtin_bit_cast(i16x4, b),
                                                     c, 0, 0, 0);
}

__device__ __forceinline__ uint4 pack_relu(const f32x4 d0, const f32x4 d1) {
    return uint4{relu2(pack2(d0[0], d0[1])), relu2(pack2(d0[2], d0[3])), relu2(pack2(d1[0], d1[1])),
                 relu2(pack2(d1[2], d1[3]))};
}

// the 8 bfloat16 starting one element before / after an aligned 16-byte block M
__device__ __forceinline__ uint4 funnel_l(const uint4 L, const uint4 M) {
    return uint4{__builtin_amdgcn_alignbit(M.x, L.w, 16), __builtin_amdgcn_alignbit(M.y, M.x, 16),
                 __builtin_amdgcn_alignbit(M.z, M.y, 16), __builtin_amdgcn_alignbit(M.w, M.z, 16)};
}
__device__ __forceinline__ uint4 funnel_r(const uint4 M, const uint4 R) {
    return uint4{__builtin_amdgcn_alignbit(M.y, M.x, 16), __builtin_amdgcn_alignbit(M.z, M.y, 16),
                 __builtin_amdgcn_alignbit(M.w, M.z, 16), __builtin_amdgcn_alignbit(R.x, M.w, 16)};
}

__device__ __forceinline__ uint4 lds16(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- packing

__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ p, uint16_t *__restrict__ out) {
    const int e = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (e < kPackHalfs) {
        float v = 0.f;
        if (e < kPF2) {
            const int h = e >> 8, lane = (e >> 2) & 63, j = e & 3, m = lane & 15, g = lane >> 4;
            if (g < 3 && j < 3) v = float((__bf16)p[kOffW1 + (16 * h + m) * 9 + 3 * g + j]) * (1.f / 64.f);
        } else if (e < kPF3) {
            const int q = e - kPF2, t = q >> 10, h = (q >> 9) & 1, lane = (q >> 3) & 63, j = q & 7;
            const int m = lane & 15, g = lane >> 4;
            v = p[kOffW2 + ((16 * h + m) * 32 + slot_channel(8 * g + j)) * 9 + t];
        } else if (e < kPB3) {
            const int q = e - kPF3, dx = q >> 9, lane = (q >> 3) & 63, j = q & 7, m = lane & 15, g = lane >> 4;
            if (m < 3) v = p[kOffW3 + slot_channel(8 * g + j) * 9 + 3 * m + dx];
        } else if (e < kPB2) {
            const int q = e - kPB3, h = q >> 8, lane = (q >> 2) & 63, j = q & 3, m = lane & 15, g = lane >> 4;
            if (g < 3 && j < 3) v = p[kOffW3 + (16 * h + m) * 9 + 3 * (2 - g) + (2 - j)];
        } else {
            const int q = e - kPB2, t = q >> 10, h = (q >> 9) & 1, lane = (q >> 3) & 63, j = q & 7;
            const int m = lane & 15, g = lane >> 4;
            v = p[kOffW2 + (slot_channel(8 * g + j) * 32 + 16 * h + m) * 9 + (8 - t)];
        }
        out[e] = bf16_bits(v);
    } else if (e < kPackHalfs + 65) {
        const int b = e - kPackHalfs;
        float *bias = reinterpret_cast<float *>(reinterpret_cast<char *>(out) + kPackBiasByte);
        bias[b] = b < 32 ? p[kOffB1 + b] : b < 64 ? p[kOffB2 + b - 32] : p[kOffB3];
    }
}

// ---------------------------------------------------------------- per-layer kernels

enum Epi { kRelu = 0, kMask = 1 };

// output rows per wave of the per-layer kernels (H is a multiple of 16): a
// tile reads kConvRows + 2 input rows, so taller tiles re-read fewer halo rows
// (16 rows: 5 % less time per training step than 4, with fewer waves per
// SIMD); the 32-channel kernels step over the input rows in phases of three
constexpr int kConvRows = 16;
static_assert((kConvRows + 2) % 3 == 0, "phases of three");

struct ConvArgs {
    const void *src;           // input: uint8 images, bf16 [n][H][W] or bf16 [n][H][W][32]
    const uint16_t *w;         // packed A operands
    const float *bias;         // nullptr: none
    const uint16_t *mask;      // kMask: activation whose sign masks the result
    uint16_t *dst;
    const uint8_t *x;          // loss epilogue: decoded images
    const uint8_t *orig;       //                originals
    float *y_out;              //                y (nullable)
    float *part;               //                per wave (sum d^2, sum g3)
    float gscale;              //                2 / pixel count
    const uint16_t *w1;        // fused layers 1 + 2: layer 1's packed A operands,
    const float *bias1;        //   its bias,
    uint16_t *dst1;            //   and where its activation a1 is written
    int H, W, strips, chunks, total;
};

struct WaveTile {
    int img, c0, y0;
};
__device__ __forceinline__ bool wave_tile(const ConvArgs &a, WaveTile &t, int &gw) {
    gw = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6));
    if (gw >= a.total) return false;
    const int per = a.strips * a.chunks;
    t.img = gw / per;
    const int r = gw - t.img * per;
    t.y0 = (r / a.strips) * kConvRows;
    t.c0 = (r % a.strips) * 16;
    return true;
}

template <int EPI>
__device__ __forceinline__ uint4 load_mask(const ConvArgs &a, int64_t pix, int g) {
    if constexpr (EPI == kMask) return *reinterpret_cast<const uint4 *>(a.mask + pix * 32 + 8 * g);
    return uint4{0u, 0u, 0u, 0u};
}

// m: the mask activation of the same pixel (kMask), loaded ahead by the caller
template <int EPI>
__device__ __forceinline__ void store32(const ConvArgs &a, int64_t pix, int g, const f32x4 d0, const f32x4 d1,
                                        const uint4 m) {
    uint4 v = {pack2(d0[0], d0[1]), pack2(d0[2], d0[3]), pack2(d1[0], d1[1]), pack2(d1[2], d1[3])};
    if constexpr (EPI == kRelu) {
        v = uint4{relu2(v.x), relu2(v.y), relu2(v.z), relu2(v.w)};
    } else {
        v = uint4{mask2(v.x, m.x), mask2(v.y, m.y), mask2(v.z, m.z), mask2(v.w, m.w)};
    }
    *reinterpret_cast<uint4 *>(a.dst + pix * 32 + 8 * g) = v;
}

__device__ __forceinline__ f32x4 bias4(const float *b, int base) {
    return b ? f32x4{b[base], b[base + 1], b[base + 2], b[base + 3]} : f32x4{0.f, 0.f, 0.f, 0.f};
}

// one input channel (uint8 images or a bfloat16 gradient map) -> 32 channels
template <bool U8, int EPI>
__global__ __launch_bounds__(256) void k_conv1(const ConvArgs a) {
    WaveTile T;
    int gw;
    if (!wave_tile(a, T, gw)) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const uint2 A0 = reinterpret_cast<const uint2 *>(a.w)[lane];
    const uint2 A1 = reinterpret_cast<const uint2 *>(a.w)[64 + lane];
    const f32x4 c0 = bias4(a.bias, 4 * g), c1 = bias4(a.bias, 16 + 4 * g);
    const int64_t plane = int64_t(T.img) * a.H * a.W;
    // the 3x3 taps of row y for this lane's slots (g, j), zero outside the image
    auto gather = [&](int y, uint16_t (&v)[3]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int sy = y + g - 1, sx = T.c0 + n + j - 1;
            v[j] = 0;
            if (g < 3 && sy >= 0 && sy < a.H && sx >= 0 && sx < a.W) {
                const int64_t q = plane + int64_t(sy) * a.W + sx;
                if constexpr (U8)
                    v[j] = bf16_bits(float(int(static_cast<const uint8_t *>(a.src)[q]) - 128));
                else
                    v[j] = static_cast<const uint16_t *>(a.src)[q];
            }
        }
    };
    uint16_t nx[3];
    gather(T.y0, nx);
    for (int yy = 0; yy < kConvRows; ++yy) {
        const int y = T.y0 + yy;
        const uint2 B = {uint32_t(nx[0]) | (uint32_t(nx[1]) << 16), uint32_t(nx[2])};
        const int64_t pix = plane + int64_t(y) * a.W + T.c0 + n;
        const uint4 m = load_mask<EPI>(a, pix, g);
        if (yy + 1 < kConvRows) gather(y + 1, nx);   // next row's loads overlap this row's work
        store32<EPI>(a, pix, g, mma16(A0, B, c0), mma16(A1, B, c1), m);
    }
}

__device__ __forceinline__ void load_row32(const ConvArgs &a, int64_t plane, int rho, int c0, int n, int g,
                                           uint4 (&B)[3]) {
    const uint16_t *src = static_cast<const uint16_t *>(a.src);
    const bool rok = rho >= 0 && rho < a.H;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int col = c0 + n + dx - 1;
        B[dx] = uint4{0u, 0u, 0u, 0u};
        if (rok && col >= 0 && col < a.W)
            B[dx] = *reinterpret_cast<const uint4 *>(src + (plane + int64_t(rho) * a.W + col) * 32 + 8 * g);
    }
}

// B: input row y0 - 1 + s, loaded by the previous step; replaced by the next row
template <int EPI, int P>
__device__ __forceinline__ void conv32_step(const ConvArgs &a, const uint4 (&F)[9][2], const f32x4 (&bv)[2],
                                            f32x4 (&acc)[3][2], uint4 (&B)[3], int s, const WaveTile &T,
                                            int64_t plane, int n, int g) {
    const uint4 Bc[3] = {B[0], B[1], B[2]};
    const int64_t pix = plane + int64_t(T.y0 + s - 2) * a.W + T.c0 + n;
    const uint4 m = s >= 2 ? load_mask<EPI>(a, pix, g) : uint4{0u, 0u, 0u, 0u};
    if (s + 1 < kConvRows + 2) load_row32(a, plane, T.y0 + s, T.c0, n, g, B);
    // input row y0-1+s feeds output rows y0+s-dy; slot of output row y is (y - y0) mod 3
    constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        acc[S0][h] = mma32(F[0][h], Bc[0], bv[h]);
        acc[S0][h] = mma32(F[1][h], Bc[1], acc[S0][h]);
        acc[S0][h] = mma32(F[2][h], Bc[2], acc[S0][h]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc[S1][h] = mma32(F[3 + dx][h], Bc[dx], acc[S1][h]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc[S2][h] = mma32(F[6 + dx][h], Bc[dx], acc[S2][h]);
    }
    if (s >= 2) store32<EPI>(a, pix, g, acc[S2][0], acc[S2][1], m);
}

// 32 channels -> 32 channels
template <int EPI>
__global__ __launch_bounds__(256) void k_conv32(const ConvArgs a) {
    // the 18 KB of packed weights are read from memory once per workgroup
    __shared__ uint4 sw[9 * 2 * 64];
    for (int i = threadIdx.x; i < 9 * 2 * 64; i += 256) sw[i] = reinterpret_cast<const uint4 *>(a.w)[i];
    __syncthreads();
    WaveTile T;
    int gw;
    if (!wave_tile(a, T, gw)) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    uint4 F[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) F[t][h] = sw[(t * 2 + h) * 64 + lane];
    const f32x4 bv[2] = {bias4(a.bias, 4 * g), bias4(a.bias, 16 + 4 * g)};
    f32x4 acc[3][2] = {};
    const int64_t plane = int64_t(T.img) * a.H * a.W;
    uint4 B[3];
    load_row32(a, plane, T.y0 - 1, T.c0, n, g, B);
    for (int s = 0; s < kConvRows + 2; s += 3) {
        conv32_step<EPI, 0>(a, F, bv, acc, B, s, T, plane, n, g);
        conv32_step<EPI, 1>(a, F, bv, acc, B, s + 1, T, plane, n, g);
        conv32_step<EPI, 2>(a, F, bv, acc, B, s + 2, T, plane, n, g);
    }
}

// Layers 1 and 2 in one pass.  Layer 2 reads layer 1's activation at three
// column shifts; here each input row of it is computed in the wave instead of
// loaded: for shift dx the lane's B operand holds the 3 x 3 taps of x around
// pixel (row, c0 + n + dx - 1) (lanes g < 3, tap row g), one mma16 per half of
// the 32 channels gives a1 there in exactly the slot layout layer 2 reads as
// its B operand, and positions outside the image are zero (layer 2's padding).
// The same products on the same operands as k_conv1, so a1 and a2 are the
// values the two kernels give; the centre shift of the tile's own rows is
// written as a1 for the backward pass.  x taps of the next input row are
// loaded one step ahead.
struct XTaps {
    uint16_t v[5];     // bf16 of x - 128 (0 outside the image) at columns c0 + n - 2 .. c0 + n + 2
};

__device__ __forceinline__ void gather_taps(const ConvArgs &a, int64_t plane, int rho, int c0, int n, int g,
                                            XTaps &t) {
    const int sy = rho + g - 1;
    const bool rok = g < 3 && sy >= 0 && sy < a.H;
    const uint8_t *src = static_cast<const uint8_t *>(a.src) + plane + int64_t(rok ? sy : 0) * a.W;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int sx = c0 + n + j - 2;
        t.v[j] = (rok && sx >= 0 && sx < a.W) ? bf16_bits(float(int(src[sx]) - 128)) : uint16_t(0);
    }
}

template <int P>
__device__ __forceinline__ void conv12_step(const ConvArgs &a, const uint4 (&F)[9][2], const uint2 (&A1)[2],
                                            const f32x4 (&b1)[2], const f32x4 (&bv)[2], f32x4 (&acc)[3][2],
                                            XTaps &X, int s, const WaveTile &T, int64_t plane, int n, int g) {
    const XTaps Xc = X;
    const int rho = T.y0 - 1 + s;
    if (s + 1 < kConvRows + 2) gather_taps(a, plane, rho + 1, T.c0, n, g, X);
    uint4 Bc[3];
    const bool rok = rho >= 0 && rho < a.H;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const uint2 B = {uint32_t(Xc.v[dx]) | (uint32_t(Xc.v[dx + 1]) << 16), uint32_t(Xc.v[dx + 2])};
        const uint4 v = pack_relu(mma16(A1[0], B, b1[0]), mma16(A1[1], B, b1[1]));
        const int col = T.c0 + n + dx - 1;
        Bc[dx] = (rok && col >= 0 && col < a.W) ? v : uint4{0u, 0u, 0u, 0u};
    }
    if (s >= 1 && s <= kConvRows)
        *reinterpret_cast<uint4 *>(a.dst1 + (plane + int64_t(rho) * a.W + T.c0 + n) * 32 + 8 * g) = Bc[1];
    const int64_t pix = plane + int64_t(T.y0 + s - 2) * a.W + T.c0 + n;
    constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        acc[S0][h] = mma32(F[0][h], Bc[0], bv[h]);
        acc[S0][h] = mma32(F[1][h], Bc[1], acc[S0][h]);
        acc[S0][h] = mma32(F[2][h], Bc[2], acc[S0][h]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc[S1][h] = mma32(F[3 + dx][h], Bc[dx], acc[S1][h]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc[S2][h] = mma32(F[6 + dx][h], Bc[dx], acc[S2][h]);
    }
    if (s >= 2) store32<kRelu>(a, pix, g, acc[S2][0], acc[S2][1], uint4{0u, 0u, 0u, 0u});
}

// Held to 3 waves per SIMD (164 VGPRs): uncapped it takes 176 and runs two,
// slower than the two separate kernels it replaces.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_conv12(const ConvArgs a) {
    __shared__ uint4 sw[9 * 2 * 64];
    for (int i = threadIdx.x; i < 9 * 2 * 64; i += 256) sw[i] = reinterpret_cast<const uint4 *>(a.w)[i];
    __syncthreads();
    WaveTile T;
    int gw;
    if (!wave_tile(a, T, gw)) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    uint4 F[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) F[t][h] = sw[(t * 2 + h) * 64 + lane];
    const uint2 A1[2] = {reinterpret_cast<const uint2 *>(a.w1)[lane], reinterpret_cast<const uint2 *>(a.w1)[64 + lane]};
    const f32x4 b1[2] = {bias4(a.bias1, 4 * g), bias4(a.bias1, 16 + 4 * g)};
    const f32x4 bv[2] = {bias4(a.bias, 4 * g), bias4(a.bias, 16 + 4 * g)};
    f32x4 acc[3][2] = {};
    const int64_t plane = int64_t(T.img) * a.H * a.W;
    XTaps X;
    gather_taps(a, plane, T.y0 - 1, T.c0, n, g, X);
    for (int s = 0; s < kConvRows + 2; s += 3) {
        conv12_step<0>(a, F, A1, b1, bv, acc, X, s, T, plane, n, g);
        conv12_step<1>(a, F, A1, b1, bv, acc, X, s + 1, T, plane, n, g);
        conv12_step<2>(a, F, A1, b1, bv, acc, X, s + 2, T, plane, n, g);
    }
}

// 32 channels -> 1 channel, residual, loss and its gradient.  A row m = dy of
// the layer-3 operand for column shift dx puts each input row's contribution
// to output row (input row + 1 - dy) in accumulator register dy; the
// registers then shift by one per input row.
__global__ __launch_bounds__(256) void k_conv_out(const ConvArgs a) {
    WaveTile T;
    int gw;
    if (!wave_tile(a, T, gw)) return;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    uint4 F[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) F[dx] = reinterpret_cast<const uint4 *>(a.w)[dx * 64 + lane];
    const float b3 = a.bias[0];
    const int64_t plane = int64_t(T.img) * a.H * a.W;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    float lsum = 0.f, gsum = 0.f;
    uint4 B[3];
    load_row32(a, plane, T.y0 - 1, T.c0, n, g, B);
    for (int s = 0; s < kConvRows + 2; ++s) {
        const uint4 Bc[3] = {B[0], B[1], B[2]};
        const int64_t pix = plane + int64_t(T.y0 + s - 2) * a.W + T.c0 + n;
        int xv = 0, ov = 0;
        if (s >= 2 && g == 0) {
            xv = a.x[pix];
            ov = a.orig[pix];
        }
        if (s + 1 < kConvRows + 2) load_row32(a, plane, T.y0 + s, T.c0, n, g, B);
        acc = mma32(F[0], Bc[0], acc);
        acc = mma32(F[1], Bc[1], acc);
        acc = mma32(F[2], Bc[2], acc);
        if (s >= 2 && g == 0) {
            const float yv = float(xv - 128) * (1.f / 64.f) + (acc[2] + b3);
            const float d = yv - float(ov - 128) * (1.f / 64.f);
            const uint16_t gb = bf16_bits(d * a.gscale);
            a.dst[pix] = gb;
            if (a.y_out) a.y_out[pix] = yv;
            lsum += d * d;
            gsum += bf16_float(gb);
        }
        acc = f32x4{0.f, acc[0], acc[1], 0.f};
    }
    lsum = wave_sum_f(lsum);
    gsum = wave_sum_f(gsum);
    if (lane == 0) {
        a.part[2 * gw] = lsum;
        a.part[2 * gw + 1] = gsum;
    }
}

// ---------------------------------------------------------------- weight gradients
//
// One workgroup (4 waves) per (image, band of 16 rows), in sub-bands of 4 rows.
// LDS tiles are channel-major: T[slot][row][column].  The activation tile has
// one halo row above and below and 8 zero columns on each side; its slot
// stride is padded so the 16 lanes of a group read 16 different bank quads.

struct WgradArgs {
    const uint16_t *g;     // output-side gradient: [n][H][W][32] (dz), or [n][H][W] (g3)
    const uint16_t *act;   // input-side activation [n][H][W][32]
    const uint8_t *x;      // decoded images (first layer)
    float *part;           // [workgroup][kParams]
    int H, W, lw, bands;   // W = 1 << lw
    int items;             // (image, 16-row band) pairs; workgroup b takes b, b + grid, ...
};

// Workgroups of the weight-gradient kernels: each loops over its (image, band)
// items in a fixed order and writes one partial row, so the partial sums the
// reduction reads are at most this many rows whatever the batch.
constexpr int kWgradGrid = 512;

// rows [row0, row0 + nrows) of a 32-channel map -> T[slot * sstride + r * rpitch + coff + px]
// (W = 1 << lw)
__device__ __forceinline__ void stage32(uint16_t *T, int sstride, int rpitch, int coff, const uint16_t *src,
                                        int img, int row0, int nrows, int H, int lw) {
    const int W = 1 << lw;
    for (int c = int(threadIdx.x); c < (nrows * 4) << lw; c += 256) {
        const int px = c & (W - 1), rest = c >> lw, q = rest & 3, r = rest >> 2;
        const int row = row0 + r;
        uint4 v = {0u, 0u, 0u, 0u};
        if (row >= 0 && row < H)
            v = *reinterpret_cast<const uint4 *>(src + ((int64_t(img) * H + row) * W + px) * 32 + 8 * q);
        uint16_t *d = T + (8 * q) * sstride + r * rpitch + coff + px;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            d[(2 * k) * sstride] = uint16_t(w[k] & 0xffffu);
            d[(2 * k + 1) * sstride] = uint16_t(w[k] >> 16);
        }
    }
}

// The same in two phases, so the global loads of the next rows can be in
// flight while the current ones are used: load into registers (at most MAXC
// 16-byte chunks per thread), later transpose them into LDS.
template <int MAXC>
struct Staged {
    uint4 v[MAXC];
};
template <int MAXC>
__device__ __forceinline__ void stage_load(Staged<MAXC> &st, const uint16_t *src, int img, int row0, int nrows,
                                           int H, int lw) {
    const int W = 1 << lw;
#pragma unroll
    for (int k = 0; k < MAXC; ++k) {
        const int c = int(threadIdx.x) + 256 * k;
        st.v[k] = uint4{0u, 0u, 0u, 0u};
        if (c < (nrows * 4) << lw) {
            const int px = c & (W - 1), rest = c >> lw, q = rest & 3, row = row0 + (rest >> 2);
            if (row >= 0 && row < H)
                st.v[k] = *reinterpret_cast<const uint4 *>(src + ((int64_t(img) * H + row) * W + px) * 32 + 8 * q);
        }
    }
}
template <int MAXC>
__device__ __forceinline__ void stage_store(const Staged<MAXC> &st, uint16_t *T, int sstride, int rpitch, int coff,
                                            int nrows, int lw) {
    const int W = 1 << lw;
#pragma unroll
    for (int k = 0; k < MAXC; ++k) {
        const int c = int(threadIdx.x) + 256 * k;
        if (c < (nrows * 4) << lw) {
            const int px = c & (W - 1), rest = c >> lw, q = rest & 3, r = rest >> 2;
            uint16_t *d = T + (8 * q) * sstride + r * rpitch + coff + px;
            const uint32_t w[4] = {st.v[k].x, st.v[k].y, st.v[k].z, st.v[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                d[(2 * j) * sstride] = uint16_t(w[j] & 0xffffu);
                d[(2 * j + 1) * sstride] = uint16_t(w[j] >> 16);
            }
        }
    }
}

__device__ __forceinline__ int dz_stride(int W) { return 4 * W + 8; }
__device__ __forceinline__ int act_pitch(int W) { return W + 16; }
__device__ __forceinline__ int act_stride(int W) { return 6 * (W + 16) + 8; }

constexpr uint32_t kOne2 = 0x3f803f80u;   // two bfloat16 ones

// dW2[o][i][t] = sum_p dz2[o][p] a1[i][p + off_t];  db2[o] = sum_p dz2[o][p].
// Wave w owns the input half ih = w % 2 for both output halves and all 9 taps
// (the activation operands it reads from LDS serve 18 products: 11 LDS reads
// for 18 MFMAs), over the 32-pixel chunks of parity ph = w / 2.  The two
// waves of one input half add their sums through LDS in a fixed order, so the
// partial row is deterministic.
constexpr int kW2Red = 80;   // floats per lane in the final exchange: 2 x 9 x 4 taps + 2 x 4 bias
__global__ __launch_bounds__(256) void k_wgrad2(const WgradArgs a) {
    extern __shared__ uint4 smem4[];
    uint16_t *sm = reinterpret_cast<uint16_t *>(smem4);
    const int W = a.W, DS = dz_stride(W), AP = act_pitch(W), AS = act_stride(W);
    uint16_t *dzT = sm, *aT = sm + 32 * DS;
    const int tid = threadIdx.x, lane = tid & 63, n = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ih = wave & 1, ph = wave >> 1;
    for (int c = tid; c < 32 * 6 * 16; c += 256) {
        const int k = c & 15, r = (c >> 4) % 6, sl = c / 96;
        aT[sl * AS + r * AP + (k < 8 ? k : W + k)] = 0;
    }
    f32x4 acc[2][9] = {};
    f32x4 accb[2] = {};
    const uint4 ones = {kOne2, kOne2, kOne2, kOne2};
    const int lcpr = a.lw - 5;   // log2 of the 32-pixel chunks per row
    for (int item = int(blockIdx.x); item < a.items; item += int(gridDim.x)) {
    const int img = item / a.bands, y0 = (item % a.bands) * 16;
    // sub-band sb + 1 is loaded into registers while sub-band sb is computed
    Staged<4> sd;   // 4 rows x 4 chunks x W <= 1024 chunks
    Staged<6> sa;   // 6 rows
    stage_load(sd, a.g, img, y0, 4, a.H, a.lw);
    stage_load(sa, a.act, img, y0 - 1, 6, a.H, a.lw);
    for (int sb = 0; sb < 4; ++sb) {
        __syncthreads();
        stage_store(sd, dzT, DS, W, 0, 4, a.lw);
        stage_store(sa, aT, AS, AP, 8, 6, a.lw);
        __syncthreads();
        if (sb + 1 < 4) {
            stage_load(sd, a.g, img, y0 + 4 * (sb + 1), 4, a.H, a.lw);
            stage_load(sa, a.act, img, y0 + 4 * (sb + 1) - 1, 6, a.H, a.lw);
        }
        for (int k = ph; k < (4 << lcpr); k += 2) {
            const int rl = k >> lcpr, px0 = (k & ((1 << lcpr) - 1)) * 32;
            const uint4 A0 = lds16(dzT + n * DS + rl * W + px0 + 8 * g);
            const uint4 A1 = lds16(dzT + (16 + n) * DS + rl * W + px0 + 8 * g);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const uint16_t *base = aT + (16 * ih + n) * AS + (rl + dy) * AP + 8 + px0 + 8 * g;
                const uint4 L = lds16(base - 8), M = lds16(base), R = lds16(base + 8);
                const uint4 Bl = funnel_l(L, M), Br = funnel_r(M, R);
                acc[0][3 * dy + 0] = mma32(A0, Bl, acc[0][3 * dy + 0]);
                acc[1][3 * dy + 0] = mma32(A1, Bl, acc[1][3 * dy + 0]);
                acc[0][3 * dy + 1] = mma32(A0, M, acc[0][3 * dy + 1]);
                acc[1][3 * dy + 1] = mma32(A1, M, acc[1][3 * dy + 1]);
                acc[0][3 * dy + 2] = mma32(A0, Br, acc[0][3 * dy + 2]);
                acc[1][3 * dy + 2] = mma32(A1, Br, acc[1][3 * dy + 2]);
            }
            if (ih == 0) {
                accb[0] = mma32(A0, ones, accb[0]);
                accb[1] = mma32(A1, ones, accb[1]);
            }
        }
    }
    __syncthreads();   // the next item restages the tiles
    }
    // pixel-parity halves: ph = 1 hands its sums over, ph = 0 adds them and writes
    float *red = reinterpret_cast<float *>(smem4) + (ih * 64 + lane) * kW2Red;
    if (ph == 1) {
#pragma unroll
        for (int oh = 0; oh < 2; ++oh) {
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[(oh * 9 + t) * 4 + i] = acc[oh][t][i];
#pragma unroll
            for (int i = 0; i < 4; ++i) red[72 + oh * 4 + i] = accb[oh][i];
        }
    }
    __syncthreads();
    if (ph == 1) return;
    float *dst = a.part + int64_t(blockIdx.x) * kParams;
    const int ii = slot_channel(16 * ih + n);
#pragma unroll
    for (int oh = 0; oh < 2; ++oh)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = slot_channel(16 * oh + 4 * g + i);
#pragma unroll
            for (int t = 0; t < 9; ++t) dst[kOffW2 + (o * 32 + ii) * 9 + t] = acc[oh][t][i] + red[(oh * 9 + t) * 4 + i];
            if (ih == 0 && n == 0) dst[kOffB2 + o] = accb[oh][i] + red[72 + oh * 4 + i];
        }
}

// dW1[o][t] = sum_p dz1[o][p] xn[p + off_t] (B column t < 9), db1 (column 9 = ones)
// The single-channel tiles are small, so wgrad1 and wgrad3 stage 8 rows at a
// time (two staging rounds per band instead of four).
constexpr int kSb1 = 8;

__global__ __launch_bounds__(256) void k_wgrad1(const WgradArgs a) {
    extern __shared__ uint4 smem4[];
    uint16_t *sm = reinterpret_cast<uint16_t *>(smem4);
    const int W = a.W, DS = kSb1 * W + 8, AP = act_pitch(W);
    uint16_t *dzT = sm, *xT = sm + 32 * DS;
    const int tid = threadIdx.x, lane = tid & 63, n = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int c = tid; c < (kSb1 + 2) * 16; c += 256) {
        const int k = c & 15, r = c >> 4;
        xT[r * AP + (k < 8 ? k : W + k)] = 0;
    }
    f32x4 acc[2] = {};
    const int tap = n < 9 ? n : 4;
    const int dy = tap / 3, dx = tap % 3;
    const int cpr = W / 32;
    // the next sub-band is loaded into registers while the current one is used
    for (int item = int(blockIdx.x); item < a.items; item += int(gridDim.x)) {
    const int img = item / a.bands, y0 = (item % a.bands) * 16;
    Staged<kSb1> sd;
    uint16_t xv[3];   // (kSb1 + 2) rows x W <= 640 values, 3 per thread
    auto load_x = [&](int r0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int c = tid + 256 * k, r = c >> a.lw, px = c & (W - 1), row = r0 - 1 + r;
            xv[k] = 0;
            if (c < (kSb1 + 2) * W && row >= 0 && row < a.H)
                xv[k] = bf16_bits(float(int(a.x[(int64_t(img) * a.H + row) * W + px]) - 128) * (1.f / 64.f));
        }
    };
    stage_load(sd, a.g, img, y0, kSb1, a.H, a.lw);
    load_x(y0);
    for (int sb = 0; sb < 16 / kSb1; ++sb) {
        __syncthreads();
        stage_store(sd, dzT, DS, W, 0, kSb1, a.lw);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int c = tid + 256 * k;
            if (c < (kSb1 + 2) * W) xT[(c >> a.lw) * AP + 8 + (c & (W - 1))] = xv[k];
        }
        __syncthreads();
        if (sb + 1 < 16 / kSb1) {
            stage_load(sd, a.g, img, y0 + kSb1 * (sb + 1), kSb1, a.H, a.lw);
            load_x(y0 + kSb1 * (sb + 1));
        }
        for (int k = wave; k < kSb1 * cpr; k += 4) {
            const int rl = k / cpr, px0 = (k % cpr) * 32;
            const uint16_t *base = xT + (rl + dy) * AP + 8 + px0 + 8 * g;
            const uint4 L = lds16(base - 8), M = lds16(base), R = lds16(base + 8);
            uint4 B = dx == 0 ? funnel_l(L, M) : dx == 1 ? M : funnel_r(M, R);
            if (n == 9) B = uint4{kOne2, kOne2, kOne2, kOne2};
            if (n > 9) B = uint4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int oh = 0; oh < 2; ++oh)
                acc[oh] = mma32(lds16(dzT + (16 * oh + n) * DS + rl * W + px0 + 8 * g), B, acc[oh]);
        }
    }
    __syncthreads();
    }
    float *red = reinterpret_cast<float *>(smem4);   // [32][10]
    for (int w = 0; w < 4; ++w) {
        if (wave == w && n < 10)
#pragma unroll
            for (int oh = 0; oh < 2; ++oh)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float &r = red[slot_channel(16 * oh + 4 * g + i) * 10 + n];
                    r = (w ? r : 0.f) + acc[oh][i];
                }
        __syncthreads();
    }
    float *dst = a.part + int64_t(blockIdx.x) * kParams;
    for (int e = tid; e < 320; e += 256) {
        const int o = e / 10, c = e % 10;
        dst[c < 9 ? kOffW1 + o * 9 + c : kOffB1 + o] = red[e];
    }
}

// dW3[i][t] = sum_q g3[q - off_t] a2[i][q]: A row m = tap takes g3 shifted by -off_t
__global__ __launch_bounds__(256) void k_wgrad3(const WgradArgs a) {
    extern __shared__ uint4 smem4[];
    uint16_t *sm = reinterpret_cast<uint16_t *>(smem4);
    const int W = a.W, DS = kSb1 * W + 8, AP = act_pitch(W);
    uint16_t *aT = sm, *gT = sm + 32 * DS;
    const int tid = threadIdx.x, lane = tid & 63, n = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int c = tid; c < (kSb1 + 2) * 16; c += 256) {
        const int k = c & 15, r = c >> 4;
        gT[r * AP + (k < 8 ? k : W + k)] = 0;
    }
    f32x4 acc[2] = {};
    const int tap = n < 9 ? n : 4;
    const int dy = tap / 3, dx = tap % 3;
    const int cpr = W / 32;
    for (int item = int(blockIdx.x); item < a.items; item += int(gridDim.x)) {
    const int img = item / a.bands, y0 = (item % a.bands) * 16;
    Staged<kSb1> sa;
    uint16_t gv[3];
    auto load_g = [&](int r0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int c = tid + 256 * k, r = c >> a.lw, px = c & (W - 1), row = r0 - 1 + r;
            gv[k] = 0;
            if (c < (kSb1 + 2) * W && row >= 0 && row < a.H) gv[k] = a.g[(int64_t(img) * a.H + row) * W + px];
        }
    };
    stage_load(sa, a.act, img, y0, kSb1, a.H, a.lw);
    load_g(y0);
    for (int sb = 0; sb < 16 / kSb1; ++sb) {
        __syncthreads();
        stage_store(sa, aT, DS, W, 0, kSb1, a.lw);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int c = tid + 256 * k;
            if (c < (kSb1 + 2) * W) gT[(c >> a.lw) * AP + 8 + (c & (W - 1))] = gv[k];
        }
        __syncthreads();
        if (sb + 1 < 16 / kSb1) {
            stage_load(sa, a.act, img, y0 + kSb1 * (sb + 1), kSb1, a.H, a.lw);
            load_g(y0 + kSb1 * (sb + 1));
        }
        for (int k = wave; k < kSb1 * cpr; k += 4) {
            const int rl = k / cpr, px0 = (k % cpr) * 32;
            const uint16_t *base = gT + (rl + 2 - dy) * AP + 8 + px0 + 8 * g;
            const uint4 L = lds16(base - 8), M = lds16(base), R = lds16(base + 8);
            uint4 A = dx == 0 ? funnel_r(M, R) : dx == 1 ? M : funnel_l(L, M);
            if (n > 8) A = uint4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int ih = 0; ih < 2; ++ih)
                acc[ih] = mma32(A, lds16(aT + (16 * ih + n) * DS + rl * W + px0 + 8 * g), acc[ih]);
        }
    }
    __syncthreads();
    }
    float *red = reinterpret_cast<float *>(smem4);   // [32 channels][9 taps]
    for (int w = 0; w < 4; ++w) {
        if (wave == w)
#pragma unroll
            for (int ih = 0; ih < 2; ++ih)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int t = 4 * g + i;
                    if (t < 9) {
                        float &r = red[slot_channel(16 * ih + n) * 9 + t];
                        r = (w ? r : 0.f) + acc[ih][i];
                    }
                }
        __syncthreads();
    }
    float *dst = a.part + int64_t(blockIdx.x) * kParams;
    for (int e = tid; e < 288; e += 256) dst[kOffW3 + e] = red[e];
}

// fixed-order sums over workgroups: deterministic gradient and loss.  Blocks
// below kRedParamBlocks take kRedCols consecutive weight-gradient entries (128
// contiguous bytes of every partial row); their kRedGroups row groups each sum
// every kRedGroups-th partial row, with up to 16 loads of a thread in flight
// together (one round at 512 partial rows), and the group sums are added in a
// fixed order.  The last two blocks sum the per-wave partials of the
// loss-gradient kernel (b3's gradient, then the loss) with all threads and a
// fixed-order tree.
constexpr int kRedThreads = 1024;
constexpr int kRedCols = 32, kRedGroups = kRedThreads / kRedCols;
constexpr int kRedParamBlocks = (kOffB3 + kRedCols - 1) / kRedCols;

// Adam's state and hyper-parameters (c1, c2: the bias corrections of the step)
struct AdamArgs {
    float *p, *m, *v;
    float lr, b1, b2, eps, c1, c2;
};

__device__ __forceinline__ void adam_one(const AdamArgs &a, int i, float g) {
    const float mm = a.b1 * a.m[i] + (1.f - a.b1) * g;
    const float vv = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
    a.m[i] = mm;
    a.v[i] = vv;
    a.p[i] -= a.lr * (mm * a.c1) / (sqrtf(vv * a.c2) + a.eps);
}

// ADAM: the thread that completes a gradient entry also applies the update
template <bool ADAM>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const float *__restrict__ part, int n_wg,
                                                        const float *__restrict__ part3, int n_w3, float inv_count,
                                                        float *__restrict__ grad, float *__restrict__ loss,
                                                        const AdamArgs ad) {
    __shared__ float sm[kRedThreads];
    const int tid = threadIdx.x;
    if (int(blockIdx.x) >= kRedParamBlocks) {
        const int k = int(blockIdx.x) == kRedParamBlocks ? 1 : 0;   // 1: b3 gradient, 0: loss
        float s = 0.f;
        for (int w = tid; w < n_w3; w += kRedThreads) s += part3[2 * w + k];
        sm[tid] = s;
        __syncthreads();
        for (int h = kRedThreads / 2; h > 0; h >>= 1) {
            if (tid < h) sm[tid] += sm[tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            if (k) {
                grad[kOffB3] = sm[0];
                if constexpr (ADAM) adam_one(ad, kOffB3, sm[0]);
            } else if (loss) {
                *loss = sm[0] * inv_count;
            }
        }
        return;
    }
    const int c = tid % kRedCols, q = tid / kRedCols;
    const int p = int(blockIdx.x) * kRedCols + c;
    float s = 0.f;
    if (p < kOffB3) {
        int w = q;
        for (; w + 15 * kRedGroups < n_wg; w += 16 * kRedGroups) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = part[int64_t(w + k * kRedGroups) * kParams + p];
#pragma unroll
            for (int k = 0; k < 16; ++k) s += v[k];
        }
        for (; w < n_wg; w += kRedGroups) s += part[int64_t(w) * kParams + p];
    }
    sm[tid] = s;
    __syncthreads();
    if (q == 0 && p < kOffB3) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < kRedGroups; ++k) t += sm[k * kRedCols + c];
        grad[p] = t;
        if constexpr (ADAM) adam_one(ad, p, t);
    }
}

__global__ __launch_bounds__(256) void k_adam(const AdamArgs a, const float *__restrict__ grad) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i < kParams) adam_one(a, i, grad[i]);
}

// ---------------------------------------------------------------- fused inference

constexpr int kStripOut = 14;   // output columns per wave (16 lanes, one halo column each side)
constexpr int kChunkRows = 32;  // output rows per wave item

struct ApplyPlane {
    int64_t off;
    int32_t H, W, pitch, strips, chunks, item_start;
};

struct ApplyArgs {
    const uint8_t *in;
    uint8_t *out;
    const uint8_t *orig;
    unsigned long long *sse;
    const uint16_t *w;
    const float *bias;
    int64_t fs_in, fs_out, fs_orig;
    int32_t n_frames, n_planes, items_per_frame, pad;
    ApplyPlane pl[kMaxPlanes];
};

struct Ctx {
    uint4 F2[9][2];
    uint2 F1[2];
    uint4 F3[3];
    f32x4 b1v[2], b2v[2];
    float b3;
    f32x4 acc2[3][2];
    f32x4 acc3;
    uint32_t word;        // lanes 0..19: x - 128 of rows (rho-2 .. rho+1) in bytes 0..3
    uint32_t pre[3];      // prefetched x rows (same lane layout)
    uint32_t opre[3];     // prefetched original pixels of future output rows
    uint32_t sse;
    // uniform row pointers at the column of lane offset 0, advanced by one row per step
    const uint8_t *xrow;  // x row loaded next (row rho + 4 of the step)
    const uint8_t *orow;  // original row loaded next (row rho + 1)
    uint8_t *drow;        // output row written next (row rho - 2)
    // interior tiles: row 0 of the plane at column ccol - 2 (x) / ccol (original);
    // border tiles: the plane origins (columns are clamped per lane)
    const uint8_t *src, *org;
    int64_t pitch;
    int H, W, y0, ccol, lsh, n, g;
    int xoff, ooff, bsrc;   // lane offsets of the x window, the output column, its owner lane
    bool ok1[3], ok2;       // border tiles: a1 columns (per shift) and the a2 column inside the plane
    bool okout, xok;        // this lane writes an output pixel; its x column is inside the plane
};

// x row `row` (EDGE: any row; zero outside the image) at column ccol - 2 + min(lane, 19)
template <bool EDGE>
__device__ __forceinline__ uint32_t load_x(Ctx &c, int row) {
    if constexpr (!EDGE) {
        const uint32_t v = c.xrow[c.xoff];
        c.xrow += c.pitch;
        return (v - 128u) & 0xffu;
    } else {
        const int rr = min(max(row, 0), c.H - 1);
        const uint32_t v = c.src[int64_t(rr) * c.pitch + c.xoff];
        return (c.xok && row == rr) ? (v - 128u) & 0xffu : 0u;
    }
}
template <bool EDGE>
__device__ __forceinline__ uint32_t load_o(Ctx &c, int row) {
    if constexpr (!EDGE) {
        const uint32_t v = c.orow[c.ooff];
        c.orow += c.pitch;
        return v;
    } else {
        const int rr = min(max(row, 0), c.H - 1);
        return c.org[int64_t(rr) * c.pitch + c.ooff];
    }
}

// One a1 row step.  P = s mod 3 (accumulator slots), A2: an a2 row completes,
// EMIT: an output row completes, PREF: prefetch for step s + 3.
template <bool EDGE, int P, bool A2, bool EMIT, bool PREF>
__device__ __forceinline__ void apply_step(Ctx &c, int s) {
    const int rho = c.y0 - 2 + s;   // a1 row of this step
    {
        const uint32_t cur = c.pre[P];
        if constexpr (PREF) c.pre[P] = load_x<EDGE>(c, rho + 4);
        c.word = (c.word >> 8) | (cur << 24);
    }
    // original pixel of output row rho - 2; prefetch the one three steps on
    const uint32_t o = c.opre[P];
    if constexpr (PREF) c.opre[P] = load_o<EDGE>(c, rho + 1);
    // layer-1 B operands: slot (g, j) = xn at (rho + g - 1, column + dx + j - 1)
    float v[5];
    int w2 = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int w = __shfl(int(c.word), c.n + q, 64);
        if (q == 2) w2 = w;
        v[q] = float(int(uint32_t(w) << c.lsh) >> 24);
    }
    uint4 B2[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const uint2 B1 = {pack2(v[dx], v[dx + 1]), pack2(v[dx + 2], 0.f)};
        uint4 u = pack_relu(mma16(c.F1[0], B1, c.b1v[0]), mma16(c.F1[1], B1, c.b1v[1]));
        if constexpr (EDGE) {
            if (rho < 0 || rho >= c.H || !c.ok1[dx]) u = uint4{0u, 0u, 0u, 0u};
        }
        B2[dx] = u;
    }
    // layer 2: a1 row rho feeds a2 rows rho + 1 - dy, slot (a2 row - y0 + 1) mod 3
    constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        c.acc2[S0][h] = mma32(c.F2[0][h], B2[0], c.b2v[h]);
        c.acc2[S0][h] = mma32(c.F2[1][h], B2[1], c.acc2[S0][h]);
        c.acc2[S0][h] = mma32(c.F2[2][h], B2[2], c.acc2[S0][h]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) c.acc2[S1][h] = mma32(c.F2[3 + dx][h], B2[dx], c.acc2[S1][h]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) c.acc2[S2][h] = mma32(c.F2[6 + dx][h], B2[dx], c.acc2[S2][h]);
    }
    if constexpr (!A2) return;
    // a2 row rho - 1 is complete
    uint4 u = pack_relu(c.acc2[S2][0], c.acc2[S2][1]);
    if constexpr (EDGE) {
        const int r2 = rho - 1;
        if (r2 < 0 || r2 >= c.H || !c.ok2) u = uint4{0u, 0u, 0u, 0u};
    }
    const uint4 uL = {uint32_t(__builtin_amdgcn_update_dpp(0, int(u.x), 0x111, 0xf, 0xf, true)),
                      uint32_t(__builtin_amdgcn_update_dpp(0, int(u.y), 0x111, 0xf, 0xf, true)),
                      uint32_t(__builtin_amdgcn_update_dpp(0, int(u.z), 0x111, 0xf, 0xf, true)),
                      uint32_t(__builtin_amdgcn_update_dpp(0, int(u.w), 0x111, 0xf, 0xf, true))};
    const uint4 uR = {uint32_t(__builtin_amdgcn_update_dpp(0, int(u.x), 0x101, 0xf, 0xf, true)),
                      uint32_t(__builtin_amdgcn_update_dpp(0, int(u.y), 0x101, 0xf, 0xf, true)),
                      uint32_t(__builtin_amdgcn_update_dpp(0, int(u.z), 0x101, 0xf, 0xf, true)),
                      uint32_t(__builtin_amdgcn_update_dpp(0, int(u.w), 0x101, 0xf, 0xf, true))};
    c.acc3 = mma32(c.F3[0], uL, c.acc3);
    c.acc3 = mma32(c.F3[1], u, c.acc3);
    c.acc3 = mma32(c.F3[2], uR, c.acc3);
    if constexpr (EMIT) {
        // output row rho - 2 is complete (register 2)
        const int yo = rho - 2;
        bool live = c.okout;
        if constexpr (EDGE) live = live && yo < c.H;
        const float xc = float((int(uint32_t(w2) << 24) >> 24) + 128);   // byte 0: row rho - 2
        const float val = __builtin_rintf(fmaf(64.f, c.acc3[2] + c.b3, xc));
        const uint32_t pix = uint32_t(fminf(fmaxf(val, 0.f), 255.f));
        if constexpr (EDGE) {
            if (live) c.drow[int64_t(yo - c.y0) * c.pitch + c.ooff] = uint8_t(pix);
        } else {
            // every lane stores the byte of column ccol + ooff, taken from the
            // lane that owns it: lanes sharing an address write the same value
            c.drow[c.ooff] = uint8_t(__shfl(int(pix), c.bsrc, 64));
            c.drow += c.pitch;
        }
        const int d = int(pix) - int(o);
        c.sse += live ? uint32_t(d * d) : 0u;
    }
    c.acc3 = f32x4{0.f, c.acc3[0], c.acc3[1], 0.f};
}

// The 36 steps of one 32-row item: four prologue steps, nine unrolled triples,
// five epilogue steps (the last three need no prefetch).  Row pointers (c.drow
// set by the caller) advance one row per load / store on the interior path.
template <bool EDGE>
__device__ __forceinline__ void apply_item(Ctx &c) {
    c.sse = 0;
    c.acc3 = f32x4{0.f, 0.f, 0.f, 0.f};
    // x rows y0-4 .. y0-2 in bytes 1..3; rows y0-1 .. y0+1 prefetched for steps 0..2
    c.xrow = c.src + int64_t(c.y0 - 4) * c.pitch;
    c.orow = c.org + int64_t(c.y0 - 4) * c.pitch;
    const uint32_t r0 = load_x<EDGE>(c, c.y0 - 4);
    const uint32_t r1 = load_x<EDGE>(c, c.y0 - 3);
    const uint32_t r2 = load_x<EDGE>(c, c.y0 - 2);
    c.word = (r0 << 8) | (r1 << 16) | (r2 << 24);
#pragma unroll
    for (int k = 0; k < 3; ++k) c.pre[k] = load_x<EDGE>(c, c.y0 - 1 + k);
#pragma unroll
    for (int k = 0; k < 3; ++k) c.opre[k] = load_o<EDGE>(c, c.y0 - 4 + k);
    apply_step<EDGE, 0, false, false, true>(c, 0);
    apply_step<EDGE, 1, false, false, true>(c, 1);
    apply_step<EDGE, 2, true, false, true>(c, 2);
    apply_step<EDGE, 0, true, false, true>(c, 3);
    for (int s = 4; s < 31; s += 3) {
        apply_step<EDGE, 1, true, true, true>(c, s);
        apply_step<EDGE, 2, true, true, true>(c, s + 1);
        apply_step<EDGE, 0, true, true, true>(c, s + 2);
    }
    apply_step<EDGE, 1, true, true, true>(c, 31);
    apply_step<EDGE, 2, true, true, true>(c, 32);
    apply_step<EDGE, 0, true, true, false>(c, 33);
    apply_step<EDGE, 1, true, true, false>(c, 34);
    apply_step<EDGE, 2, true, true, false>(c, 35);
}
static_assert(kChunkRows == 32, "the step schedule of apply_item covers 36 steps");

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_apply(const ApplyArgs a) {
    const int lane = threadIdx.x & 63;
    Ctx c;
    c.n = lane & 15;
    c.g = lane >> 4;
    c.lsh = c.g < 3 ? 16 - 8 * c.g : 0;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) c.F2[t][h] = reinterpret_cast<const uint4 *>(a.w + kPF2)[(t * 2 + h) * 64 + lane];
#pragma unroll
    for (int h = 0; h < 2; ++h) c.F1[h] = reinterpret_cast<const uint2 *>(a.w + kPF1)[h * 64 + lane];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) c.F3[dx] = reinterpret_cast<const uint4 *>(a.w + kPF3)[dx * 64 + lane];
    c.b1v[0] = bias4(a.bias, 4 * c.g);
    c.b1v[1] = bias4(a.bias, 16 + 4 * c.g);
    c.b2v[0] = bias4(a.bias + 32, 4 * c.g);
    c.b2v[1] = bias4(a.bias + 32, 16 + 4 * c.g);
    c.b3 = a.bias[64];

    const int total = a.n_frames * a.items_per_frame;
    const int nw = int(gridDim.x) * 4;
    for (int item = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6)); item < total;
         item += nw) {
        const int f = item / a.items_per_frame;
        const int w = item - f * a.items_per_frame;
        int p = 0;
        while (p + 1 < a.n_planes && w >= a.pl[p + 1].item_start) ++p;
        const ApplyPlane &P = a.pl[p];
        const int q = w - P.item_start;
        const int chunk = q / P.strips, strip = q - chunk * P.strips;
        c.H = P.H;
        c.W = P.W;
        c.pitch = P.pitch;
        c.y0 = chunk * kChunkRows;
        c.ccol = strip * kStripOut - 1;   // column of lane n = 0 for a2 and the output
        const bool interior = c.y0 >= 3 && c.y0 + 34 < c.H && c.ccol - 2 >= 0 && c.ccol + 17 < c.W;
        const int xl = min(lane, 19);
        const int on = min(max(c.n, 1), kStripOut);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int col = c.ccol + c.n + dx - 1;
            c.ok1[dx] = col >= 0 && col < c.W;
        }
        c.ok2 = c.ccol + c.n >= 0 && c.ccol + c.n < c.W;
        c.okout = c.g == 0 && c.n >= 1 && c.n <= kStripOut && c.ccol + c.n < c.W;
        const uint8_t *fsrc = a.in + int64_t(f) * a.fs_in + P.off;
        // without originals the loads read the input (valid memory) and no error is kept
        const uint8_t *forg = a.orig ? a.orig + int64_t(f) * a.fs_orig + P.off : fsrc;
        uint8_t *fdst = a.out + int64_t(f) * a.fs_out + P.off;
        if (interior) {
            // row pointers at column ccol - 2 (x) and ccol (orig, out); lane offsets in range
            c.xoff = xl;
            c.ooff = on;
            c.bsrc = on;
            c.src = fsrc + (c.ccol - 2);
            c.org = forg + c.ccol;
            c.xok = true;
            c.drow = fdst + c.ccol + int64_t(c.y0) * c.pitch;
            apply_item<false>(c);
        } else {
            // clamped columns; out-of-image values are zeroed by the masks
            const int xc = c.ccol - 2 + xl;
            c.xok = xc >= 0 && xc < c.W;
            c.xoff = min(max(xc, 0), c.W - 1);
            c.ooff = min(max(c.ccol + on, 0), c.W - 1);
            c.src = fsrc;
            c.org = forg;
            c.drow = fdst + int64_t(c.y0) * c.pitch;
            apply_item<true>(c);
        }
        if (a.sse) {
            uint32_t e = c.sse;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
            if (lane == 0 && e) atomicAdd(a.sse + int64_t(f) * a.n_planes + p, (unsigned long long)e);
        }
    }
}

__global__ void k_zero_sse(unsigned long long *p, int n) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i < n) p[i] = 0ull;
}

// keep rule + fallback copy: one block per (row over all planes, frame)
__global__ __launch_bounds__(256) void k_select(const unsigned long long *__restrict__ sf,
                                                const unsigned long long *__restrict__ sr, const uint8_t *plain,
                                                int64_t fs_plain, uint8_t *out, int64_t fs_out, uint8_t *keep,
                                                const ApplyArgs a) {
    const int f = blockIdx.y;
    unsigned long long tf = 0, tr = 0;
    for (int p = 0; p < a.n_planes; ++p) {
        tf += sf[int64_t(f) * a.n_planes + p];
        tr += sr[int64_t(f) * a.n_planes + p];
    }
    const bool k = tf <= tr;
    if (keep && blockIdx.x == 0 && threadIdx.x == 0) keep[f] = k ? 1 : 0;
    if (k) return;
    int row = blockIdx.x, p = 0;
    while (p + 1 < a.n_planes && row >= a.pl[p].H) {
        row -= a.pl[p].H;
        ++p;
    }
    const ApplyPlane &P = a.pl[p];
    const uint8_t *s = plain + int64_t(f) * fs_plain + P.off + int64_t(row) * P.pitch;
    uint8_t *d = out + int64_t(f) * fs_out + P.off + int64_t(row) * P.pitch;
    for (int c = int(threadIdx.x); c < P.W / 8; c += 256)
        reinterpret_cast<uint2 *>(d)[c] = reinterpret_cast<const uint2 *>(s)[c];
}

// ---------------------------------------------------------------- host side

struct WsLayout {
    int64_t packed, a1, a2, dz2, dz1, g3, part, part3, grad, total;
    int n_wg, n_w3;
};

int64_t up256(int64_t v) { return (v + 255) & ~int64_t(255); }

adct_status train_dims(int n, int H, int W) {
    if (n < 1) return fail(ADCT_ERANGE, "n must be >= 1");
    if (H < 16 || H % 16 || (W != 32 && W != 64))
        return fail(ADCT_EDIM, "training images need H a multiple of 16 and W = 32 or 64");
    if (int64_t(n) * H * W > (int64_t(1) << 31) / 64) return fail(ADCT_ERANGE, "batch too large");
    return ADCT_OK;
}

WsLayout layout(int n, int H, int W) {
    WsLayout L;
    const int64_t px = int64_t(n) * H * W;
    L.n_wg = std::min(n * (H / 16), kWgradGrid);
    L.n_w3 = n * (W / 16) * (H / kConvRows);
    int64_t o = 0;
    L.packed = o; o += up256(kPackBytes);
    L.a1 = o; o += up256(px * 64);
    L.a2 = o; o += up256(px * 64);
    L.dz2 = o; o += up256(px * 64);
    L.dz1 = o; o += up256(px * 64);
    L.g3 = o; o += up256(px * 2);
    L.part = o; o += up256(int64_t(L.n_wg) * kParams * 4);
    L.part3 = o; o += up256(int64_t(L.n_w3) * 8);
    L.grad = o; o += up256(int64_t(kParams) * 4);
    L.total = o;
    return L;
}

size_t wgrad_lds(int W) {
    const size_t stage2 = size_t(32 * (4 * W + 8) + 32 * (6 * (W + 16) + 8)) * 2;        // wgrad2
    const size_t stage13 = size_t(32 * (kSb1 * W + 8) + (kSb1 + 2) * (W + 16)) * 2;      // wgrad1, wgrad3
    const size_t red2 = size_t(2 * 64 * kW2Red) * 4;                                       // wgrad2's exchange
    return std::max(std::max(std::max(stage2, stage13), size_t(32 * 10) * 4), red2);
}

// Adam's bias corrections for a step (host side, float64)
adct_status adam_args(float *params, float *m, float *v, int step, float lr, float beta1, float beta2,
                      float eps, AdamArgs *a) {
    if (step < 1) return fail(ADCT_ERANGE, "step counts from 1");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(ADCT_ERANGE, "need lr >= 0, beta1 and beta2 in [0, 1), eps > 0");
    a->p = params;
    a->m = m;
    a->v = v;
    a->lr = lr;
    a->b1 = beta1;
    a->b2 = beta2;
    a->eps = eps;
    a->c1 = float(1.0 / (1.0 - std::pow(double(beta1), step)));
    a->c2 = float(1.0 / (1.0 - std::pow(double(beta2), step)));
    return ADCT_OK;
}

// adam: null for the gradient alone, else the update is applied by the reduction
adct_status launch_grad(const float *params, const uint8_t *recon, const uint8_t *orig, int n, int H, int W,
                        char *ws, float *grad, float *loss, float *y_out, const AdamArgs *adam, hipStream_t s) {
    const WsLayout L = layout(n, H, W);
    uint16_t *packed = reinterpret_cast<uint16_t *>(ws + L.packed);
    const float *bias = reinterpret_cast<const float *>(ws + L.packed + kPackBiasByte);
    uint16_t *a1 = reinterpret_cast<uint16_t *>(ws + L.a1), *a2 = reinterpret_cast<uint16_t *>(ws + L.a2);
    uint16_t *dz2 = reinterpret_cast<uint16_t *>(ws + L.dz2), *dz1 = reinterpret_cast<uint16_t *>(ws + L.dz1);
    uint16_t *g3 = reinterpret_cast<uint16_t *>(ws + L.g3);
    float *part = reinterpret_cast<float *>(ws + L.part), *part3 = reinterpret_cast<float *>(ws + L.part3);

    hipLaunchKernelGGL(k_pack, dim3((kPackHalfs + 65 + 255) / 256), dim3(256), 0, s, params, packed);
    ConvArgs c{};
    c.H = H;
    c.W = W;
    c.strips = W / 16;
    c.chunks = H / kConvRows;
    c.total = n * c.strips * c.chunks;
    const dim3 grid((c.total + 3) / 4), blk(256);
    ConvArgs c2 = c;   // layers 1 and 2 (a1 written for the backward pass)
    c2.src = recon; c2.w = packed + kPF2; c2.bias = bias + 32; c2.dst = a2;
    c2.w1 = packed + kPF1; c2.bias1 = bias; c2.dst1 = a1;
    hipLaunchKernelGGL(k_conv12, grid, blk, 0, s, c2);
    ConvArgs c3 = c;   // layer 3 + loss
    c3.src = a2; c3.w = packed + kPF3; c3.bias = bias + 64; c3.dst = g3; c3.x = recon; c3.orig = orig;
    c3.y_out = y_out; c3.part = part3; c3.gscale = float(2.0 / (double(n) * H * W));
    hipLaunchKernelGGL(k_conv_out, grid, blk, 0, s, c3);
    ConvArgs d3 = c;   // input gradient of layer 3, masked by a2
    d3.src = g3; d3.w = packed + kPB3; d3.mask = a2; d3.dst = dz2;
    hipLaunchKernelGGL((k_conv1<false, kMask>), grid, blk, 0, s, d3);
    ConvArgs d2 = c;   // input gradient of layer 2, masked by a1
    d2.src = dz2; d2.w = packed + kPB2; d2.mask = a1; d2.dst = dz1;
    hipLaunchKernelGGL(k_conv32<kMask>, grid, blk, 0, s, d2);

    WgradArgs wa{};
    wa.part = part;
    wa.H = H;
    wa.W = W;
    wa.lw = W == 64 ? 6 : 5;
    wa.bands = H / 16;
    wa.items = n * wa.bands;
    const size_t lds = wgrad_lds(W);
    WgradArgs w3 = wa;
    w3.g = g3; w3.act = a2;
    hipLaunchKernelGGL(k_wgrad3, dim3(L.n_wg), blk, lds, s, w3);
    WgradArgs w2 = wa;
    w2.g = dz2; w2.act = a1;
    hipLaunchKernelGGL(k_wgrad2, dim3(L.n_wg), blk, lds, s, w2);
    WgradArgs w1 = wa;
    w1.g = dz1; w1.x = recon;
    hipLaunchKernelGGL(k_wgrad1, dim3(L.n_wg), blk, lds, s, w1);
    const float inv_count = float(1.0 / (double(n) * H * W));
    if (adam)
        hipLaunchKernelGGL(k_reduce<true>, dim3(kRedParamBlocks + 2), dim3(kRedThreads), 0, s, part, L.n_wg, part3, L.n_w3,
                           inv_count, grad, loss, *adam);
    else
        hipLaunchKernelGGL(k_reduce<false>, dim3(kRedParamBlocks + 2), dim3(kRedThreads), 0, s, part, L.n_wg, part3, L.n_w3,
                           inv_count, grad, loss, AdamArgs{});
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

adct_status launch_adam(float *params, float *m, float *v, const float *grad, int step, float lr, float beta1,
                        float beta2, float eps, hipStream_t s) {
    AdamArgs ad;
    if (adct_status st = adam_args(params, m, v, step, lr, beta1, beta2, eps, &ad)) return st;
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, ad, grad);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

adct_status apply_args(const uint8_t *frames, int64_t fs, int n_frames, const adct_plane *planes, int n_planes,
                       uint8_t *out, int64_t fs_out, ApplyArgs *a) {
    if (!frames || !planes || !out) return fail(ADCT_EINVAL, "frames, planes and out are required");
    if (n_frames < 1) return fail(ADCT_ERANGE, "n_frames must be >= 1");
    if (n_planes < 1 || n_planes > kMaxPlanes) return fail(ADCT_ERANGE, "n_planes must be in [1, 4]");
    if (frames == out) return fail(ADCT_EINVAL, "the filter cannot work in place");
    *a = ApplyArgs{};
    int items = 0;
    for (int p = 0; p < n_planes; ++p) {
        const adct_plane &q = planes[p];
        if (q.H < 1 || q.W < 1 || q.pitch < q.W || q.offset < 0)
            return fail(ADCT_EDIM, "plane needs H, W >= 1, pitch >= W, offset >= 0");
        ApplyPlane &P = a->pl[p];
        P.off = q.offset;
        P.H = q.H;
        P.W = q.W;
        P.pitch = q.pitch;
        P.strips = (q.W + kStripOut - 1) / kStripOut;
        P.chunks = (q.H + kChunkRows - 1) / kChunkRows;
        P.item_start = items;
        items += P.strips * P.chunks;
    }
    if (int64_t(items) * n_frames > (int64_t(1) << 31) - 1) return fail(ADCT_ERANGE, "too many frames");
    a->in = frames;
    a->out = out;
    a->fs_in = fs;
    a->fs_out = fs_out;
    a->n_frames = n_frames;
    a->n_planes = n_planes;
    a->items_per_frame = items;
    return ADCT_OK;
}

int apply_grid() {
    static thread_local int cached_dev = -1, grid = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != cached_dev) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_apply, 256, 0) != hipSuccess) return 0;
        grid = std::max(1, per) * cus;
        cached_dev = dev;
    }
    return grid;
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

int64_t adct_filter_packed_bytes(void) { return kPackBytes; }

adct_status adct_filter_pack(const float *params, void *packed, adct_stream_t stream) {
    if (!params || !packed) return fail(ADCT_EINVAL, "params and packed are required");
    hipLaunchKernelGGL(k_pack, dim3((kPackHalfs + 65 + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), params, static_cast<uint16_t *>(packed));
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

int64_t adct_filter_workspace_bytes(int n, int H, int W) {
    if (train_dims(n, H, W)) return -1;
    return layout(n, H, W).total;
}

adct_status adct_filter_grad(const float *params, const uint8_t *recon, const uint8_t *orig, int n, int H, int W,
                             void *workspace, int64_t ws_bytes, float *grad, float *loss, float *y_out,
                             adct_stream_t stream) {
    if (!params || !recon || !orig || !workspace || !grad)
        return fail(ADCT_EINVAL, "params, recon, orig, workspace and grad are required");
    if (adct_status st = train_dims(n, H, W)) return st;
    if (ws_bytes < layout(n, H, W).total) return fail(ADCT_ECAP, "workspace too small");
    return launch_grad(params, recon, orig, n, H, W, static_cast<char *>(workspace), grad, loss, y_out, nullptr,
                       reinterpret_cast<hipStream_t>(stream));
}

adct_status adct_filter_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                             float beta1, float beta2, float eps, adct_stream_t stream) {
    if (!params || !m || !v || !grad) return fail(ADCT_EINVAL, "params, m, v and grad are required");
    return launch_adam(params, m, v, grad, step, lr, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream));
}

adct_status adct_filter_train_step(float *params, float *m, float *v, int step, float lr, float beta1, float beta2,
                                   float eps, const uint8_t *recon, const uint8_t *orig, int n, int H, int W,
                                   void *workspace, int64_t ws_bytes, float *loss, adct_stream_t stream) {
    if (!params || !m || !v || !recon || !orig || !workspace)
        return fail(ADCT_EINVAL, "params, m, v, recon, orig and workspace are required");
    if (adct_status st = train_dims(n, H, W)) return st;
    const WsLayout L = layout(n, H, W);
    if (ws_bytes < L.total) return fail(ADCT_ECAP, "workspace too small");
    AdamArgs ad;
    if (adct_status st = adam_args(params, m, v, step, lr, beta1, beta2, eps, &ad)) return st;
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *grad = reinterpret_cast<float *>(ws + L.grad);
    return launch_grad(params, recon, orig, n, H, W, ws, grad, loss, nullptr, &ad, s);
}

adct_status adct_filter_apply(const void *packed, const uint8_t *frames, int64_t frame_stride, int n_frames,
                              const adct_plane *planes, int n_planes, uint8_t *out, int64_t frame_stride_out,
                              const uint8_t *orig, int64_t frame_stride_orig, uint64_t *sse,
                              adct_stream_t stream) {
    if (!packed) return fail(ADCT_EINVAL, "packed weights are required");
    if (reinterpret_cast<uintptr_t>(packed) % 16) return fail(ADCT_EDIM, "packed weights must be 16-byte aligned");
    ApplyArgs a;
    if (adct_status st = apply_args(frames, frame_stride, n_frames, planes, n_planes, out, frame_stride_out, &a))
        return st;
    if (sse && !orig) return fail(ADCT_EINVAL, "sse needs orig");
    a.orig = orig;
    a.fs_orig = frame_stride_orig;
    a.sse = reinterpret_cast<unsigned long long *>(sse);
    a.w = static_cast<const uint16_t *>(packed);
    a.bias = reinterpret_cast<const float *>(static_cast<const char *>(packed) + kPackBiasByte);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (sse) {
        const int nz = n_frames * n_planes;
        hipLaunchKernelGGL(k_zero_sse, dim3((nz + 255) / 256), dim3(256), 0, s, a.sse, nz);
    }
    const int grid = apply_grid();
    if (grid < 1) return fail(ADCT_EDEVICE, "cannot size the filter grid");
    const int64_t items = int64_t(a.items_per_frame) * n_frames;
    hipLaunchKernelGGL(k_apply, dim3(int(std::min<int64_t>(grid, (items + 3) / 4))), dim3(256), 0, s, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

adct_status adct_filter_select(const uint64_t *sse_filtered, const uint64_t *sse_reference, int n_frames,
                               int n_planes, const uint8_t *plain, int64_t frame_stride_plain,
                               const adct_plane *planes, uint8_t *out, int64_t frame_stride_out, uint8_t *keep,
                               adct_stream_t stream) {
    if (!sse_filtered || !sse_reference || !plain) return fail(ADCT_EINVAL, "sse arrays and plain are required");
    ApplyArgs a;
    if (adct_status st = apply_args(plain, frame_stride_plain, n_frames, planes, n_planes, out, frame_stride_out, &a))
        return st;
    int rows = 0;
    for (int p = 0; p < n_planes; ++p) {
        const adct_plane &q = planes[p];
        if (q.W % 8 || q.pitch % 8 || q.offset % 8)
            return fail(ADCT_EDIM, "select copies 8-byte words: W, pitch and offset must be multiples of 8");
        rows += q.H;
    }
    if (frame_stride_plain % 8 || frame_stride_out % 8 || reinterpret_cast<uintptr_t>(plain) % 8 ||
        reinterpret_cast<uintptr_t>(out) % 8)
        return fail(ADCT_EDIM, "frame buffers and strides must be 8-byte aligned");
    hipLaunchKernelGGL(k_select, dim3(rows, n_frames), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       reinterpret_cast<const unsigned long long *>(sse_filtered),
                       reinterpret_cast<const unsigned long long *>(sse_reference), plain, frame_stride_plain, out,
                       frame_stride_out, keep, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

// ---------------------------------------------------------------- checkpoint
//
// Host blob: 64-byte header, then float32 params [kParams] and, when flag bit 0
// is set, the Adam moments m and v [kParams] each.  Header: magic "ADCTFILT",
// uint32 version (1), uint32 parameter count, uint32 flags, int32 Adam step,
// uint64 FNV-1a hash of the payload bytes, zero padding.

namespace {
constexpr char kCkMagic[8] = {'A', 'D', 'C', 'T', 'F', 'I', 'L', 'T'};
constexpr uint32_t kCkVersion = 1;
struct CkHeader {
    char magic[8];
    uint32_t version, count, flags;
    int32_t step;
    uint64_t hash;
    uint8_t pad[32];
};
static_assert(sizeof(CkHeader) == 64, "checkpoint header is 64 bytes");

uint64_t fnv1a(const uint8_t *p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}
}  // namespace

int64_t adct_filter_checkpoint_bytes(int with_moments) {
    return int64_t(sizeof(CkHeader)) + int64_t(with_moments ? 3 : 1) * kParams * int64_t(sizeof(float));
}

adct_status adct_filter_save(const float *params, const float *m, const float *v, int step, void *blob,
                             int64_t blob_bytes, adct_stream_t stream) {
    if (!params || !blob) return fail(ADCT_EINVAL, "params and blob are required");
    if ((m == nullptr) != (v == nullptr)) return fail(ADCT_EINVAL, "m and v go together");
    const int with = m != nullptr;
    const int64_t need = adct_filter_checkpoint_bytes(with);
    if (blob_bytes < need) return fail(ADCT_ECAP, "blob is smaller than adct_filter_checkpoint_bytes()");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *payload = static_cast<uint8_t *>(blob) + sizeof(CkHeader);
    const size_t part = size_t(kParams) * sizeof(float);
    ADCT_HIP(hipMemcpyAsync(payload, params, part, hipMemcpyDeviceToHost, s));
    if (with) {
        ADCT_HIP(hipMemcpyAsync(payload + part, m, part, hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipMemcpyAsync(payload + 2 * part, v, part, hipMemcpyDeviceToHost, s));
    }
    ADCT_HIP(hipStreamSynchronize(s));
    CkHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kCkMagic, 8);
    h.version = kCkVersion;
    h.count = kParams;
    h.flags = uint32_t(with);
    h.step = step;
    h.hash = fnv1a(payload, size_t(need) - sizeof(CkHeader));
    memcpy(blob, &h, sizeof(h));
    return ADCT_OK;
}

adct_status adct_filter_load(const void *blob, int64_t blob_bytes, float *params, float *m, float *v, int *step,
                             adct_stream_t stream) {
    if (!blob || !params) return fail(ADCT_EINVAL, "blob and params are required");
    if ((m == nullptr) != (v == nullptr)) return fail(ADCT_EINVAL, "m and v go together");
    if (blob_bytes < int64_t(sizeof(CkHeader))) return fail(ADCT_EDIM, "blob is shorter than its header");
    CkHeader h;
    memcpy(&h, blob, sizeof(h));
    if (memcmp(h.magic, kCkMagic, 8) != 0) return fail(ADCT_EINVAL, "not a post-filter checkpoint");
    if (h.version != kCkVersion || h.count != uint32_t(kParams) || h.flags > 1)
        return fail(ADCT_EINVAL, "checkpoint version or parameter count does not match this library");
    const int64_t need = adct_filter_checkpoint_bytes(int(h.flags));
    if (blob_bytes != need) return fail(ADCT_EDIM, "blob size does not match its header");
    const uint8_t *payload = static_cast<const uint8_t *>(blob) + sizeof(CkHeader);
    if (fnv1a(payload, size_t(need) - sizeof(CkHeader)) != h.hash)
        return fail(ADCT_EINVAL, "checkpoint payload is corrupted (hash mismatch)");
    if (m && !h.flags) return fail(ADCT_EINVAL, "the checkpoint holds no optimiser moments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t part = size_t(kParams) * sizeof(float);
    ADCT_HIP(hipMemcpyAsync(params, payload, part, hipMemcpyHostToDevice, s));
    if (m) {
        ADCT_HIP(hipMemcpyAsync(m, payload + part, part, hipMemcpyHostToDevice, s));
        ADCT_HIP(hipMemcpyAsync(v, payload + 2 * part, part, hipMemcpyHostToDevice, s));
    }
    ADCT_HIP(hipStreamSynchronize(s));
    if (step) *step = h.step;
    return ADCT_OK;
}

}  // extern "C"
