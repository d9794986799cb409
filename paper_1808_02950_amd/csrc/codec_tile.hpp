// Device helpers shared by the 8x8 codec kernels (built-in matrices and
// matrices given at run time): the wave's tile of 64 blocks, its loads, row
// packing with squared-error dot products, rounding and the quantiser.
#pragma once

#include <algorithm>

#include "adct_internal.hpp"
#include "wave.hpp"

namespace adct {
namespace {

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int byte_of(uint32_t w, int i) { return int((w >> (8 * i)) & 0xffu); }

// round-half-to-even of a float64 to int32 (|x| < 2^31): adding 1.5 * 2^52
// leaves the rounded integer in the low word of the sum.
__device__ __forceinline__ int rne_i32(double x) {
    return __double2loint(x + 6755399441055744.0);
}

__device__ __forceinline__ int clamp255(int v) { return min(max(v, 0), 255); }

// n / d for 0 <= n < 2^31 and a wave-uniform d, from its magic pair (m, s).
__device__ __forceinline__ int udiv_magic(int n, uint32_t m, int s) {
    return s < 0 ? n : int(__umulhi(uint32_t(n), m) >> s);
}

// round-half-away(Y / d) for d = step mu (a class n_k n_l = mu^2, where Y / d can
// be an exact half), in float32: floor((2|Y| + d + 1/2) / (2d)) is the rounded
// magnitude, and its argument |Y| / d + (d + 1/2) / (2d) lies at least 1/(4d)
// from an integer, while c1 = 1/d and c2 = (d + 1/2)/(2d) in float32 and one fma
// err by less than (2 x + 1) 2^-24 with x < |Y| / d + 1 -- below 1/(4d) whenever
// |Y| + d < 2^21 (the host requires 2^20).  The sign of Y is copied onto the
// quotient, whose truncation toward zero is then the signed level.
__device__ __forceinline__ int quant_rational_f(int y, float c1, float c2) {
    const float yf = float(y);
    const float x = fmaf(fabsf(yf), c1, c2);
    const float xs = __int_as_float(int((__float_as_uint(x) & 0x7fffffffu) | (__float_as_uint(yf) & 0x80000000u)));
    return int(xs);
}

// round-half-away(Y / d), d = step * mu, for the classes where n_k n_l = mu^2
// (Y / d can be an exact half): floor((2|Y| + d) / (2d)) from a float estimate
// corrected in exact integer arithmetic (2|Y| + d < 2^24 is checked on the host).
__device__ __forceinline__ int quant_rational(int y, int step, int mu, float inv_2mu, float inv_step) {
    const int ay = y < 0 ? -y : y;
    const int d = step * mu;                                  // wave-uniform
    const int d2 = d + d;
    const int num = 2 * ay + d;
    int q = int(float(num) * inv_2mu * inv_step);
    const int rem = num - __mul24(q, d2);
    q += (rem >= d2) ? 1 : 0;
    q -= (rem < 0) ? 1 : 0;
    return y < 0 ? -q : q;
}

// round-half-away(Y s_k s_l / step) where s_k s_l = 1/sqrt(n_k n_l) is
// irrational: the quotient is never an exact half (its nearest half is > 1e-9
// away for |Y| < 2^16, far above the float64 error), so round-half-to-even of
// the float64 product gives the same integer.
__device__ __forceinline__ int quant_irrational(int y, double skl, double inv_step) {
    return rne_i32(double(y) * skl * inv_step);
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) { return wave_sum_u32(v); }

// A wave's unit of work: 64 consecutive blocks of one plane of one frame.
struct Tile {
    int f, p;            // frame, plane (wave-uniform)
    int b;               // block index inside the plane (per lane)
    bool active;
    uint32_t in_off, out_off;
};

__device__ __forceinline__ Tile tile_of(const CodecArgs &a, int gw, int lane) {
    Tile t;
    t.f = udiv_magic(gw, a.wpf_m, a.wpf_s);
    const int w = gw - t.f * a.waves_per_frame;
    int p = 0;
    while (p + 1 < a.n_planes && w >= a.pl[p + 1].wave_start) ++p;
    t.p = p;
    const PlaneArg &P = a.pl[p];
    const int b0 = (w - P.wave_start) * 64;             // first block of the wave
    const int by0 = udiv_magic(b0, P.nbx_m, P.nbx_s);
    const int bx0 = b0 - by0 * P.nbx;
    t.b = b0 + lane;
    t.active = t.b < P.nblocks;
    int by, bx;
    if (P.nbx >= 64) {                                   // at most one row change
        bx = bx0 + lane;
        by = by0;
        if (bx >= P.nbx) {
            bx -= P.nbx;
            ++by;
        }
    } else {
        by = t.b / P.nbx;
        bx = t.b - by * P.nbx;
    }
    if (!t.active) by = bx = 0;
    t.in_off = __umul24(uint32_t(8 * by), uint32_t(P.pitch_in)) + uint32_t(8 * bx);
    t.out_off = __umul24(uint32_t(8 * by), uint32_t(P.pitch_out)) + uint32_t(8 * bx);
    return t;
}

__device__ __forceinline__ void load_tile(const CodecArgs &a, const Tile &t, uint32_t (&pix)[8][2]) {
    const PlaneArg &P = a.pl[t.p];
    const uint8_t *src = a.in + int64_t(t.f) * a.fs_in + P.in_off + t.in_off;
    // inactive lanes point at block (0, 0) of the plane: the load stays in
    // bounds and its result is never stored or scored
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const u32x2 v = __builtin_nontemporal_load((const u32x2 *)(src + x * P.pitch_in));
        pix[x][0] = v.x;
        pix[x][1] = v.y;
    }
}

// As emit_row, for a row of rounded values that still need clipping to
// [0, 255] (|q| < 2^15): pairs of values as int16 halves, one saturating pack
// per pair, two pairs per word.
__device__ __forceinline__ u32x2 emit_row_sat(const int (&q)[8], uint32_t w0, uint32_t w1,
                                              uint32_t &sq, uint32_t &cross) {
    uint32_t b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        b[i] = sat_pk_u8_i16(__builtin_amdgcn_perm(uint32_t(q[2 * i + 1]), uint32_t(q[2 * i]), 0x05040100u));
    u32x2 out;
    out.x = b[0] | (b[1] << 16);
    out.y = b[2] | (b[3] << 16);
    sq = __builtin_amdgcn_udot4(out.x, out.x, sq, false);
    sq = __builtin_amdgcn_udot4(out.y, out.y, sq, false);
    sq = __builtin_amdgcn_udot4(w0, w0, sq, false);
    sq = __builtin_amdgcn_udot4(w1, w1, sq, false);
    cross = __builtin_amdgcn_udot4(out.x, w0, cross, false);
    cross = __builtin_amdgcn_udot4(out.y, w1, cross, false);
    return out;
}

// Pack a reconstructed row (q in [0, 255]) into bytes and accumulate the two
// dot-product sums whose combination is the squared error:
// sum (q - a)^2 = [sum q^2 + sum a^2] - 2 sum q a.
__device__ __forceinline__ u32x2 emit_row(const int (&q)[8], uint32_t w0, uint32_t w1,
                                          uint32_t &sq, uint32_t &cross) {
    const uint32_t r01 = uint32_t(q[0]) | (uint32_t(q[1]) << 16);
    const uint32_t r23 = uint32_t(q[2]) | (uint32_t(q[3]) << 16);
    const uint32_t r45 = uint32_t(q[4]) | (uint32_t(q[5]) << 16);
    const uint32_t r67 = uint32_t(q[6]) | (uint32_t(q[7]) << 16);
    u32x2 out;
    out.x = __builtin_amdgcn_perm(r23, r01, 0x06040200u);
    out.y = __builtin_amdgcn_perm(r67, r45, 0x06040200u);
    sq = __builtin_amdgcn_udot4(out.x, out.x, sq, false);
    sq = __builtin_amdgcn_udot4(out.y, out.y, sq, false);
    sq = __builtin_amdgcn_udot4(w0, w0, sq, false);
    sq = __builtin_amdgcn_udot4(w1, w1, sq, false);
    cross = __builtin_amdgcn_udot4(out.x, w0, cross, false);
    cross = __builtin_amdgcn_udot4(out.y, w1, cross, false);
    return out;
}

// Persistent grid: as many 4-wave workgroups as the device keeps resident
// (occupancy x CUs), never more than there are tiles.
template <class K>
adct_status persistent_grid(K kernel, int total_waves, int *grid) {
    static thread_local int cached_dev = -1, cus = 0;
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    if (dev != cached_dev) {
        ADCT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cached_dev = dev;
    }
    int per_cu = 0;
    ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0));
    if (per_cu < 1) per_cu = 1;
    const int knob = codec_wgs_per_cu();
    if (knob > 0) per_cu = std::min(per_cu, knob);
    const int64_t want = (int64_t(total_waves) + 3) / 4;
    *grid = knob < 0 ? int(want) : int(std::min<int64_t>(want, int64_t(per_cu) * cus));
    return ADCT_OK;
}

}  // namespace
}  // namespace adct
