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

namespace adct {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

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

struct DTile {
    int f, p, b;
    bool active;
    uint32_t in_off, out_off;   // byte offset of the block's top-left pixel
};

__device__ __forceinline__ DTile dtile_of(const DctArgs &a, int gw, int n) {
    DTile t;
    t.f = gw / a.waves_per_frame;
    const int w = gw - t.f * a.waves_per_frame;
    int p = 0;
    while (p + 1 < a.n_planes && w >= a.pl[p + 1].wave_start) ++p;
    t.p = p;
    const PlaneArg &P = a.pl[p];
    t.b = (w - P.wave_start) * 16 + n;
    t.active = t.b < P.nblocks;
    const int bb = t.active ? t.b : 0;
    const int by = bb / P.nbx;
    const int bx = bb - by * P.nbx;
    t.in_off = __umul24(uint32_t(8 * by), uint32_t(P.pitch_in)) + uint32_t(8 * bx);
    t.out_off = __umul24(uint32_t(8 * by), uint32_t(P.pitch_out)) + uint32_t(8 * bx);
    return t;
}

// ONE: r <= 16, a single coefficient tile: every operand of K a lane needs
// (16 forward, 16 inverse) is read from LDS once into registers.
template <int MODE, bool ONE>
__global__ __launch_bounds__(256) void k_dct(const DctArgs a) {
    __shared__ float kf[64 * 64];
    __shared__ float ki[64 * 64];
    for (int i = threadIdx.x; i < 64 * 64; i += 256) {
        const int c = i >> 6, p = i & 63;
        const int kc = kZZ[c] >> 3, lc = kZZ[c] & 7;
        const float v = a.C[8 * kc + (p >> 3)] * a.C[8 * lc + (p & 7)];
        kf[fwd_addr(c, p)] = v;
        ki[inv_addr(p, c)] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int total = a.n_frames * a.waves_per_frame;
    const int nct = ONE ? 1 : (a.r + 15) >> 4;             // coefficient tiles
    float kfr[16], kir[16];
    if constexpr (ONE) {
#pragma unroll
        for (int s = 0; s < 16; ++s) kfr[s] = kf[fwd_addr(n, 16 * (s >> 2) + 4 * g + (s & 3))];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) kir[4 * t + s] = ki[inv_addr(16 * t + n, 4 * g + s)];
    }
    for (int gw = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
         gw < total; gw += int(gridDim.x) * 4) {
        const DTile T = dtile_of(a, gw, n);
        const PlaneArg &P = a.pl[T.p];
        const int64_t gblk = int64_t(T.f) * a.blocks_per_frame + P.block_off + T.b;

        // ---- the lane's 16 pixels: rows 2t + g/2, columns 4(g%2) .. + 3
        uint32_t px[4] = {0u, 0u, 0u, 0u};
        if constexpr (MODE != kDecode) {
            const uint8_t *src = a.in + int64_t(T.f) * a.fs_in + P.in_off + T.in_off +
                                 (g >> 1) * P.pitch_in + 4 * (g & 1);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                px[t] = __builtin_nontemporal_load((const uint32_t *)(src + 2 * t * P.pitch_in));
        }

        f32x4 acc[4] = {};                                  // inverse accumulators, pixel tiles
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
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = 16 * ct + 4 * g + i;
                float v = coef[i];
                if (c >= a.r) v = 0.f;
                if constexpr (MODE != kDecode) {
                    if (T.active && c < a.r) {
                        if (a.coef_f) a.coef_f[gblk * a.r + c] = v;
                        if (a.step) {
                            const float q = copysignf(floorf(fabsf(v) * a.inv_step + 0.5f), v);
                            if (a.coef_q) a.coef_q[gblk * a.r + c] = int16_t(q);
                            v = q * float(a.step);
                        }
                    } else if (a.step) {
                        v = 0.f;
                    }
                }
                coef[i] = v;
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
        if constexpr (MODE == kEncode) continue;

        // ---- round, clip, store 4 pixels per pixel tile, squared error
        uint32_t sq = 0, cross = 0;
        uint8_t *dst = a.out ? a.out + int64_t(T.f) * a.fs_out + P.out_off + T.out_off +
                                   (g >> 1) * P.pitch_out + 4 * (g & 1)
                             : nullptr;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t word = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float r = __builtin_amdgcn_fmed3f(rintf(acc[t][i]), 0.f, 255.f);
                word |= uint32_t(r) << (8 * i);
            }
            if (T.active && dst) __builtin_nontemporal_store(word, (uint32_t *)(dst + 2 * t * P.pitch_out));
            if constexpr (MODE == kEvaluate) {
                sq = __builtin_amdgcn_udot4(word, word, sq, false);
                sq = __builtin_amdgcn_udot4(px[t], px[t], sq, false);
                cross = __builtin_amdgcn_udot4(word, px[t], cross, false);
            }
        }
        if constexpr (MODE == kEvaluate) {
            unsigned e = T.active ? sq - 2u * cross : 0u;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
            if (lane == 0 && e) atomicAdd(a.sse + int64_t(T.f) * a.n_planes + T.p, (unsigned long long)e);
        }
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

template <int M>
adct_status launch_dct_mode(const DctArgs &a, int total_waves, hipStream_t s) {
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
