// Exact-DCT comparator on the matrix cores (gfx950, v_mfma_f32_16x16x4f32).
//
// The 2-D DCT of an 8x8 block is the dense contraction B = C A C^T; written
// over the 64 pixels of a block it is one matrix product
//     B_c = sum_p K[c][p] A_p,   K[c][p] = C[k_c][x_p] C[l_c][y_p]
// (c a zig-zag coefficient with row/column frequencies (k_c, l_c), p a pixel at
// (x_p, y_p)), and the inverse is A_p = sum_c K[c][p] B'_c.  A wave handles 16
// blocks: the forward product is (16 coefficients) x (64 pixels) x (16 blocks)
// per tile of coefficients, the inverse (16 pixels) x (16 coefficients) x (16
// blocks) per tile of pixels, both in FP32 on the MFMA units.
//
// Lane layouts of v_mfma_f32_16x16x4f32 (K = 4 per instruction):
//   A operand  lane l -> row l % 16, k-slot l / 16
//   B operand  lane l -> column l % 16, k-slot l / 16
//   D (4 regs) lane l -> rows 4 (l / 16) + i, column l % 16
// Lane l = 16 g + n works on block n.  It loads the 16 pixels of block n at rows
// 2t + g/2, columns 4 (g%2) + v (t, v = 0..3): exactly the pixels the inverse
// product leaves in its D registers, so nothing moves between lanes.  The k
// index of each product is permuted per step so that every operand a lane needs
// is one it already holds:
//   forward step s: lane (n, g) feeds its own pixel number s;
//   inverse step s: lane (n, g) feeds coefficient 16 ct + 4 g + s, which is
//                   element s of its forward result.
#include <algorithm>

#include "adct_internal.hpp"
#include "wave.hpp"

namespace adct {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Bank-conflict-free LDS layouts of K (64 x 64 floats each):
//  forward reads  (c = 16 ct + n, p with p % 16 = 4 g + s % 4, p / 16 = s / 4)
//  inverse reads  (p = 16 t + n,  c = 16 ct + 4 g + s)
// Within each read the 64 lanes hit 64 distinct banks.
__device__ __forceinline__ int fwd_addr(int c, int p) {
    const int grp = (c >> 4) * 16 + (p >> 4) * 4 + (p & 3);
    return grp * 64 + ((p & 15) >> 2) * 16 + (c & 15);
}
__device__ __forceinline__ int inv_addr(int p, int c) {
    const int grp = (c >> 4) * 16 + (p >> 4) * 4 + (c & 3);
    return grp * 64 + ((c & 15) >> 2) * 16 + (p & 15);
}

// K[c][p] = C[k][x] C[l][y] as a float32 product, except for (k, l) in
// {0, 4}^2: there a_0 = 1/sqrt(8) and a_4 cos((2n+1) pi / 4) = +-1/sqrt(8), so
// every entry is exactly +-1/8.  Using the exact value keeps those four
// coefficients exact sums over 8, so their quantiser ties (B / step exactly
// half a step) are decided as the quantiser defines them.
__device__ __forceinline__ float k_entry(const DctArgs &a, int k, int l, int x, int y) {
    const float v = a.C[8 * k + x] * a.C[8 * l + y];
    return ((k & 3) == 0 && (l & 3) == 0) ? copysignf(0.125f, v) : v;
}

struct DTile {
    int f, p, b;
    bool active;
    uint32_t in_off, out_off;   // byte offset of the block's top-left pixel
};

// n / d for 0 <= n < 2^31 from the magic pair of a wave-uniform d.
__device__ __forceinline__ int udiv_u31(int n, uint32_t m, int s) {
    return s < 0 ? n : int(__umulhi(uint32_t(n), m) >> s);
}

// Tile gw of the launch: frame and plane are wave-uniform; the wave's first
// block comes from two multiply-high divisions, and lane n's block is at most
// one block-row further when the plane is at least 16 blocks wide.
__device__ __forceinline__ DTile dtile_of(const DctArgs &a, int gw, int n) {
    DTile t;
    t.f = udiv_u31(gw, a.wpf_m, a.wpf_s);
    const int w = gw - t.f * a.waves_per_frame;
    int p = 0;
    while (p + 1 < a.n_planes && w >= a.pl[p + 1].wave_start) ++p;
    t.p = p;
    const PlaneArg &P = a.pl[p];
    const int b0 = (w - P.wave_start) * 16;
    const int by0 = udiv_u31(b0, P.nbx_m, P.nbx_s);
    const int bx0 = b0 - by0 * P.nbx;
    t.b = b0 + n;
    t.active = t.b < P.nblocks;
    int by, bx;
    if (P.nbx >= 16) {
        bx = bx0 + n;
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

// the lane's 16 pixels: rows 2t + g/2, columns 4(g%2) .. + 3 (inactive lanes
// read block (0, 0) of the plane, in bounds; the values are never used)
// (a wave-uniform plane base plus a 32-bit lane offset, so the loads take the
// scalar-base addressing form)
__device__ __forceinline__ void load_dtile(const DctArgs &a, const DTile &T, int g, uint32_t (&px)[4]) {
    const PlaneArg &P = a.pl[T.p];
    const uint8_t *base = a.in + int64_t(T.f) * a.fs_in + P.in_off;
    const uint32_t off = T.in_off + __umul24(uint32_t(g >> 1), uint32_t(P.pitch_in)) + 4u * uint32_t(g & 1);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        px[t] = __builtin_nontemporal_load((const uint32_t *)(base + (off + 2u * uint32_t(t) * uint32_t(P.pitch_in))));
}

// one 16-block tile: forward, zonal retention (+ quantiser), inverse, round,
// clip, store, squared error
template <int MODE, bool ONE>
__device__ __forceinline__ void process_dtile(const DctArgs &a, const DTile &T, const uint32_t (&px)[4],
                                              const float *kf, const float *ki, const float (&kfr)[16],
                                              const float (&kir)[16], int n, int g, int lane) {
    const PlaneArg &P = a.pl[T.p];
    const int64_t gblk = int64_t(T.f) * a.blocks_per_frame + P.block_off + T.b;
    const bool store_coef = (a.coef_f != nullptr) | (a.coef_q != nullptr);   // wave-uniform
    const int nct = ONE ? 1 : (a.r + 15) >> 4;             // coefficient tiles
    f32x4 acc[4] = {};                                      // inverse accumulators, pixel tiles
    for (int ct = 0; ct < nct; ++ct) {
        f32x4 coef = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE != kDecode) {
            // forward: coef[c = 16ct + 4g + i] for block n, as four
            // independent accumulation chains (one per pixel row pair)
            f32x4 part[4] = {};
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int p = 16 * (s >> 2) + 4 * g + (s & 3);
                const float av = ONE ? kfr[s] : kf[fwd_addr(16 * ct + n, p)];
                const float bv = float((px[s >> 2] >> (8 * (s & 3))) & 0xffu);
                part[s >> 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, part[s >> 2], 0, 0, 0);
            }
            coef = (part[0] + part[1]) + (part[2] + part[3]);
        } else {
            // decode: coefficients come from memory
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = 16 * ct + 4 * g + i;
                if (T.active && c < a.r) {
                    coef[i] = a.step ? float(a.coef_q[gblk * a.r + c]) * float(a.step)
                                     : a.coef_f[gblk * a.r + c];
                }
            }
        }
        // zonal retention (+ quantiser) and coefficient output
        float qv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = 16 * ct + 4 * g + i;
            if (c >= a.r) coef[i] = 0.f;
            if constexpr (MODE != kDecode)
                if (a.step) qv[i] = copysignf(floorf(fabsf(coef[i]) * a.inv_step + 0.5f), coef[i]);
        }
        if constexpr (MODE != kDecode) {
            if (store_coef) {
                const int64_t cb = gblk * a.r + 16 * ct + 4 * g;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (T.active && 16 * ct + 4 * g + i < a.r) {
                        if (a.coef_q) a.coef_q[cb + i] = int16_t(qv[i]);
                        if (a.coef_f) a.coef_f[cb + i] = coef[i];
                    }
                }
            }
            if (a.step) {
#pragma unroll
                for (int i = 0; i < 4; ++i) coef[i] = qv[i] * float(a.step);
            }
        }
        if constexpr (MODE == kEncode) continue;
        // inverse: acc[t] (pixels 16t + 4g + i) += sum_c K[c][p] coef_c
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float av = ONE ? kir[4 * t + s] : ki[inv_addr(16 * t + n, 16 * ct + 4 * g + s)];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, coef[s], acc[t], 0, 0, 0);
            }
    }
    if constexpr (MODE == kEncode) return;

    // ---- round, clip, store 4 pixels per pixel tile, squared error: one
    // v_cvt_pk_u8_f32 per pixel rounds half to even, saturates to [0, 255] and
    // places the byte.
    uint32_t sq = 0, cross = 0;
    uint8_t *dbase = a.out ? a.out + int64_t(T.f) * a.fs_out + P.out_off : nullptr;   // wave-uniform
    const uint32_t doff = T.out_off + __umul24(uint32_t(g >> 1), uint32_t(P.pitch_out)) + 4u * uint32_t(g & 1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint32_t word = __builtin_amdgcn_cvt_pk_u8_f32(acc[t][0], 0u, 0u);
#pragma unroll
        for (int i = 1; i < 4; ++i) word = __builtin_amdgcn_cvt_pk_u8_f32(acc[t][i], uint32_t(i), word);
        if (T.active && dbase)
            __builtin_nontemporal_store(word, (uint32_t *)(dbase + (doff + 2u * uint32_t(t) * uint32_t(P.pitch_out))));
        if constexpr (MODE == kEvaluate) {
            sq = __builtin_amdgcn_udot4(word, word, sq, false);
            sq = __builtin_amdgcn_udot4(px[t], px[t], sq, false);
            cross = __builtin_amdgcn_udot4(word, px[t], cross, false);
        }
    }
    if constexpr (MODE == kEvaluate) {
        unsigned e = T.active ? sq - 2u * cross : 0u;
        e = wave_sum_u32(e);
        if (lane == 0 && e) atomicAdd(a.sse + int64_t(T.f) * a.n_planes + T.p, (unsigned long long)e);
    }
}

// ONE: r <= 16, a single coefficient tile: every operand of K a lane needs
// (16 forward, 16 inverse) is read from LDS once into registers.  Persistent:
// each wave walks tiles gw, gw + stride, ... and loads the next tile's pixels
// into one buffer while it transforms the current tile from the other.
template <int MODE, bool ONE>
__global__ __launch_bounds__(256) void k_dct(const DctArgs a) {
    __shared__ float kf[64 * 64];
    __shared__ float ki[64 * 64];
    for (int i = threadIdx.x; i < 64 * 64; i += 256) {
        const int c = i >> 6, p = i & 63;
        const int kc = kZZ[c] >> 3, lc = kZZ[c] & 7;
        const float v = k_entry(a, kc, lc, p >> 3, p & 7);
        kf[fwd_addr(c, p)] = v;
        ki[inv_addr(p, c)] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int total = a.n_frames * a.waves_per_frame;
    const int stride = int(gridDim.x) * 4;
    float kfr[16], kir[16];
    if constexpr (ONE) {
#pragma unroll
        for (int s = 0; s < 16; ++s) kfr[s] = kf[fwd_addr(n, 16 * (s >> 2) + 4 * g + (s & 3))];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) kir[4 * t + s] = ki[inv_addr(16 * t + n, 4 * g + s)];
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) kfr[s] = kir[s] = 0.f;
    }
    int gw = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    if (gw >= total) return;                                // whole wave leaves
    uint32_t pa[4] = {0u, 0u, 0u, 0u}, pb[4] = {0u, 0u, 0u, 0u};
    DTile ta = dtile_of(a, gw, n), tb = ta;
    if constexpr (MODE != kDecode) load_dtile(a, ta, g, pa);
    // the next loads are issued on every pass (a wave's last pass re-reads its
    // current tile): no branch joins paths with different loads in flight, so
    // the waits for the current tile leave the next tile's loads outstanding
    while (true) {
        int nxt = gw + stride;
        bool more = nxt < total;                            // wave-uniform
        tb = dtile_of(a, more ? nxt : gw, n);
        if constexpr (MODE != kDecode) load_dtile(a, tb, g, pb);
        process_dtile<MODE, ONE>(a, ta, pa, kf, ki, kfr, kir, n, g, lane);
        if (!more) break;
        gw = nxt;
        nxt = gw + stride;
        more = nxt < total;
        ta = dtile_of(a, more ? nxt : gw, n);
        if constexpr (MODE != kDecode) load_dtile(a, ta, g, pa);
        process_dtile<MODE, ONE>(a, tb, pb, kf, ki, kfr, kir, n, g, lane);
        if (!more) break;
        gw = nxt;
    }
}

// ---------------------------------------------------------------- split-bfloat16 form
//
// For r <= 16 with a quantiser step that is a power of two of at least 8, the
// same products run on the bfloat16 matrix cores without losing float32
// accuracy:
//  * every float32 entry of K is the exact sum of three bfloat16 terms (each
//    rounding keeps eight more bits), so K x = K1 x + K2 x + K3 x;
//  * pixels (integers below 256) are exact in bfloat16;
//  * a quantised coefficient q * step with |q| <= 255 and step = 2^e is exact
//    in bfloat16.
// Every product is therefore exact and accumulates in float32, as in the
// float32 form.  Decoding reads q from memory, where |q| may exceed 255: there
// q * step is split into two exact bfloat16 terms, the second zero for every q
// the encoder writes, so decode repeats the evaluation's sums exactly.  Lane
// l = 16 g + n works on block n:
//  forward  v_mfma_f32_16x16x32_bf16, two halves h: K slot 8 g + j is pixel
//           (row 2 g + h, column j); the lane feeds its own two block rows;
//           result rows 4 g + i = coefficients 4 g + i of block n;
//  inverse  v_mfma_f32_16x16x16_bf16 per pixel tile t: K slot 4 g + i is
//           coefficient 4 g + i, exactly the lane's forward result; result row
//           4 g + i of tile t is pixel (row 2 g + t / 2, column 4 (t % 2) + i),
//           so the lane ends with the same two block rows it loaded.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mma32(const uint4 a, const uint4 b, const f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma16(const uint2 a, const uint2 b, const f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(i16x4, a), __builtin_bit_cast(i16x4, b),
                                                     c, 0, 0, 0);
}

// two float32 -> two bfloat16 (round to nearest even)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// k = t[0] + t[1] + t[2] exactly, each term bfloat16 (as raw bits)
__device__ __forceinline__ void split3(float k, uint32_t (&t)[3]) {
    float r = k;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const __bf16 h = (__bf16)r;
        t[s] = __builtin_bit_cast(uint16_t, h);
        r -= float(h);
    }
}

// the 8 pixels of one block row (two words) as bfloat16 operand slots 0..7
__device__ __forceinline__ uint4 row_bf16(uint32_t w0, uint32_t w1) {
    uint4 r;
    r.x = pack_bf16(float(w0 & 0xffu), float((w0 >> 8) & 0xffu));
    r.y = pack_bf16(float((w0 >> 16) & 0xffu), float(w0 >> 24));
    r.z = pack_bf16(float(w1 & 0xffu), float((w1 >> 8) & 0xffu));
    r.w = pack_bf16(float((w1 >> 16) & 0xffu), float(w1 >> 24));
    return r;
}

struct KOps {
    uint4 f[3][2];    // forward A operand [split][half]
    uint2 i[3][4];    // inverse A operand [split][pixel tile]
};

// the lane's operands of K, computed from C as the float32 products used by
// the float32 form
__device__ __forceinline__ void make_kops(const DctArgs &a, int lane, KOps &K) {
    const int row = lane & 15, g = lane >> 4;
    {
        const int kc = kZZ[row] >> 3, lc = kZZ[row] & 7;   // forward row = coefficient
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t e[3][8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint32_t t[3];
                split3(k_entry(a, kc, lc, 2 * g + h, j), t);
#pragma unroll
                for (int s = 0; s < 3; ++s) e[s][j] = t[s];
            }
#pragma unroll
            for (int s = 0; s < 3; ++s)
                K.f[s][h] = uint4{e[s][0] | (e[s][1] << 16), e[s][2] | (e[s][3] << 16), e[s][4] | (e[s][5] << 16),
                                  e[s][6] | (e[s][7] << 16)};
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {                           // inverse row = pixel of tile t
        const int x = 2 * (row >> 2) + (t >> 1), y = 4 * (t & 1) + (row & 3);
        uint32_t e[3][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int z = 4 * g + i, kc = kZZ[z] >> 3, lc = kZZ[z] & 7;
            uint32_t tt[3];
            split3(k_entry(a, kc, lc, x, y), tt);
#pragma unroll
            for (int s = 0; s < 3; ++s) e[s][i] = tt[s];
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) K.i[s][t] = uint2{e[s][0] | (e[s][1] << 16), e[s][2] | (e[s][3] << 16)};
    }
}

// the lane's two block rows 2g, 2g+1 (8 bytes each)
// (the plane's fields are read again where they are used: an empty asm makes
// the index opaque, so the compiler does not keep the fields of the eight
// tiles in flight in scalar registers, which it would spill to vector lanes)
__device__ __forceinline__ void load_rows(const DctArgs &a, const DTile &T, int g, u32x2 (&px)[2]) {
    int pi = T.p;
    asm volatile("" : "+s"(pi));
    const PlaneArg &P = a.pl[pi];
    const uint8_t *base = a.in + int64_t(T.f) * a.fs_in + P.in_off;
    const uint32_t off = T.in_off + __umul24(uint32_t(2 * g), uint32_t(P.pitch_in));
    px[0] = __builtin_nontemporal_load((const u32x2 *)(base + off));
    px[1] = __builtin_nontemporal_load((const u32x2 *)(base + (off + uint32_t(P.pitch_in))));
}

// One 16-block tile; returns the lane's squared error of its block (evaluate),
// or 0.
template <int MODE>
__device__ __forceinline__ uint32_t process_rows(const DctArgs &a, const DTile &T, const u32x2 (&px)[2],
                                                 const KOps &K, int g) {
    int pi = T.p;
    asm volatile("" : "+s"(pi));
    const PlaneArg &P = a.pl[pi];
    const int64_t cb = (int64_t(T.f) * a.blocks_per_frame + P.block_off + T.b) * a.r + 4 * g;
    const float step = float(a.step);
    float bv[4];                                            // dequantised coefficients 4g..4g+3
    if constexpr (MODE != kDecode) {
        // forward, smallest split first
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0;
        const uint4 p0 = row_bf16(px[0].x, px[0].y), p1 = row_bf16(px[1].x, px[1].y);
#pragma unroll
        for (int s = 2; s >= 0; --s) {
            c0 = mma32(K.f[s][0], p0, c0);
            c1 = mma32(K.f[s][1], p1, c1);
        }
        f32x4 coef = c0 + c1;
        // zonal retention, quantiser, coefficient output
        float qv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (4 * g + i >= a.r) coef[i] = 0.f;
            qv[i] = copysignf(floorf(fabsf(coef[i]) * a.inv_step + 0.5f), coef[i]);
            bv[i] = qv[i] * step;
        }
        if ((a.coef_f != nullptr) | (a.coef_q != nullptr)) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (T.active && 4 * g + i < a.r) {
                    if (a.coef_q) a.coef_q[cb + i] = int16_t(qv[i]);
                    if (a.coef_f) a.coef_f[cb + i] = coef[i];
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            bv[i] = (T.active && 4 * g + i < a.r) ? float(a.coef_q[cb + i]) * step : 0.f;
    }
    if constexpr (MODE == kEncode) return 0u;
    const uint2 bhi = {pack_bf16(bv[0], bv[1]), pack_bf16(bv[2], bv[3])};
    uint2 blo = {0u, 0u};
    if constexpr (MODE == kDecode) {
        float r[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t h = (i & 1) ? (i < 2 ? bhi.x : bhi.y) >> 16 : (i < 2 ? bhi.x : bhi.y) & 0xffffu;
            r[i] = bv[i] - __uint_as_float(h << 16);
        }
        blo = uint2{pack_bf16(r[0], r[1]), pack_bf16(r[2], r[3])};
    }
    // inverse, smallest split first
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 2; s >= 0; --s) {
            acc[t] = mma16(K.i[s][t], bhi, acc[t]);
            if constexpr (MODE == kDecode) acc[t] = mma16(K.i[s][t], blo, acc[t]);
        }
    }
    // round half to even with saturation to [0, 255], packed into byte i of the
    // word (one v_cvt_pk_u8_f32 per pixel), store the two rows, squared error
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint32_t v = __builtin_amdgcn_cvt_pk_u8_f32(acc[t][0], 0u, 0u);
#pragma unroll
        for (int i = 1; i < 4; ++i) v = __builtin_amdgcn_cvt_pk_u8_f32(acc[t][i], uint32_t(i), v);
        w[t] = v;
    }
    uint8_t *dbase = a.out ? a.out + int64_t(T.f) * a.fs_out + P.out_off : nullptr;   // wave-uniform
    if (T.active && dbase) {
        const uint32_t doff = T.out_off + __umul24(uint32_t(2 * g), uint32_t(P.pitch_out));
        __builtin_nontemporal_store(u32x2{w[0], w[1]}, (u32x2 *)(dbase + doff));
        __builtin_nontemporal_store(u32x2{w[2], w[3]}, (u32x2 *)(dbase + (doff + uint32_t(P.pitch_out))));
    }
    if constexpr (MODE != kEvaluate) return 0u;
    uint32_t sq = 0, cross = 0;
    const uint32_t o[4] = {px[0].x, px[0].y, px[1].x, px[1].y};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        sq = __builtin_amdgcn_udot4(w[t], w[t], sq, false);
        sq = __builtin_amdgcn_udot4(o[t], o[t], sq, false);
        cross = __builtin_amdgcn_udot4(w[t], o[t], cross, false);
    }
    return T.active ? sq - 2u * cross : 0u;
}

// A wave takes 4 consecutive 16-block tiles per pass ("group"), loads all of
// them (8 loads of 8 bytes per lane, 4 KB per wave) one group ahead, and adds
// the squared errors of tiles of one (frame, plane) before one wave sum and one
// atomic.
constexpr int kGroup = 4;

struct DGroup {
    DTile t[kGroup];
    bool live[kGroup];    // tile index inside the launch
};

__device__ __forceinline__ void group_of(const DctArgs &a, int grp, int total, int n, DGroup &G) {
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
        const int gw = grp * kGroup + q;
        G.live[q] = gw < total;
        G.t[q] = dtile_of(a, G.live[q] ? gw : total - 1, n);
    }
}

__device__ __forceinline__ void load_group(const DctArgs &a, const DGroup &G, int g, u32x2 (&px)[kGroup][2]) {
#pragma unroll
    for (int q = 0; q < kGroup; ++q) load_rows(a, G.t[q], g, px[q]);
}

template <int MODE>
__device__ __forceinline__ void process_group(const DctArgs &a, const DGroup &G, const u32x2 (&px)[kGroup][2],
                                              const KOps &K, int g, int lane) {
    uint32_t e = 0;
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
        if (G.live[q]) e += process_rows<MODE>(a, G.t[q], px[q], K, g);
        if constexpr (MODE == kEvaluate) {
            const bool last = q + 1 == kGroup || !G.live[q + 1 < kGroup ? q + 1 : q] ||
                              G.t[q + 1 < kGroup ? q + 1 : q].f != G.t[q].f ||
                              G.t[q + 1 < kGroup ? q + 1 : q].p != G.t[q].p;
            if (last && G.live[q]) {                        // wave-uniform
                uint32_t s = e;
                s = wave_sum_u32(s);
                if (lane == 0 && s)
                    atomicAdd(a.sse + int64_t(G.t[q].f) * a.n_planes + G.t[q].p, (unsigned long long)s);
                e = 0;
            }
        }
    }
}

// Held to 128 registers (4 waves per SIMD): left to itself the evaluate form
// takes 152 (3 waves) for its two groups of tile state and pixels in flight.
// The spills the cap costs (a few VGPRs to scratch, SGPRs to VGPR lanes) are
// cheaper than the lost wave: 1.78 ms against 1.97-2.10 ms on the 300-frame
// 4K stream, where 3 tiles per group at 4 waves took 1.87 ms and 2 tiles
// 2.28 ms.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_dct_bf16(const DctArgs a) {
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int total = a.n_frames * a.waves_per_frame;
    const int groups = (total + kGroup - 1) / kGroup;
    const int stride = int(gridDim.x) * 4;
    int gi = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    if (gi >= groups) return;                               // whole wave leaves
    KOps K;
    make_kops(a, lane, K);
    u32x2 pa[kGroup][2] = {}, pb[kGroup][2] = {};
    DGroup ga, gb;
    group_of(a, gi, total, n, ga);
    if constexpr (MODE != kDecode) load_group(a, ga, g, pa);
    // the next group's loads are issued on every pass (a wave's last pass
    // re-reads its current group)
    while (true) {
        int nxt = gi + stride;
        bool more = nxt < groups;                           // wave-uniform
        group_of(a, more ? nxt : gi, total, n, gb);
        if constexpr (MODE != kDecode) load_group(a, gb, g, pb);
        process_group<MODE>(a, ga, pa, K, g, lane);
        if (!more) break;
        gi = nxt;
        nxt = gi + stride;
        more = nxt < groups;
        group_of(a, more ? nxt : gi, total, n, ga);
        if constexpr (MODE != kDecode) load_group(a, ga, g, pa);
        process_group<MODE>(a, gb, pb, K, g, lane);
        if (!more) break;
        gi = nxt;
    }
}

template <int M, bool ONE>
adct_status launch_dct_kernel(const DctArgs &a, int total_waves, hipStream_t s) {
    static thread_local int cached_dev = -1, cus = 0;
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    if (dev != cached_dev) {
        ADCT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cached_dev = dev;
    }
    int per_cu = 0;
    ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dct<M, ONE>, 256, 0));
    if (per_cu < 1) per_cu = 1;
    const int64_t want = (int64_t(total_waves) + 3) / 4;
    const int grid = int(std::min<int64_t>(want, int64_t(per_cu) * cus));
    hipLaunchKernelGGL((k_dct<M, ONE>), dim3(grid), dim3(256), 0, s, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

// the split-bfloat16 form: r <= 16 and a power-of-two step of at least 8, so
// that every quantised level the encoder writes has |q| <= 255 (decoding a
// quantised stream also needs the levels, which it reads as int16)
bool bf16_form(const DctArgs &a) {
    return a.r <= 16 && a.step >= 8 && (a.step & (a.step - 1)) == 0;
}

template <int M>
adct_status launch_dct_bf16(const DctArgs &a, int total_waves, hipStream_t s) {
    static thread_local int cached_dev = -1, cus = 0;
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    if (dev != cached_dev) {
        ADCT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cached_dev = dev;
    }
    int per_cu = 0;
    ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dct_bf16<M>, 256, 0));
    if (per_cu < 1) per_cu = 1;
    const int64_t groups = (int64_t(total_waves) + kGroup - 1) / kGroup;
    const int64_t want = (groups + 3) / 4;
    const int grid = int(std::min<int64_t>(want, int64_t(per_cu) * cus));
    hipLaunchKernelGGL((k_dct_bf16<M>), dim3(grid), dim3(256), 0, s, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

template <int M>
adct_status launch_dct_mode(const DctArgs &a, int total_waves, hipStream_t s) {
    if (bf16_form(a) && (M != kDecode || a.coef_q)) return launch_dct_bf16<M>(a, total_waves, s);
    return a.r <= 16 ? launch_dct_kernel<M, true>(a, total_waves, s) : launch_dct_kernel<M, false>(a, total_waves, s);
}

}  // namespace

adct_status launch_dct(Mode mode, const DctArgs &a, int total_waves, hipStream_t s) {
    if (total_waves <= 0) return ADCT_OK;
    if (mode == kEncode) return launch_dct_mode<kEncode>(a, total_waves, s);
    if (mode == kDecode) return launch_dct_mode<kDecode>(a, total_waves, s);
    return launch_dct_mode<kEvaluate>(a, total_waves, s);
}

}  // namespace adct
