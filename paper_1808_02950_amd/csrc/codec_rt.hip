// Blockwise 8x8 transform coding with an integer matrix given at run time
// (Sec. 6.1.1 with the T that the greedy search of Eq. (6) returns, or any
// other T with orthogonal rows), and the float-coefficient decode of the
// built-in matrices.
//
// The tiling is that of the built-in codec (one lane per 8x8 block, a wave per
// 64 consecutive blocks), without its persistent grid.  What changes is the
// arithmetic: nothing about T is known at compile time, so both passes are
// plain 8-term products with wave-uniform entries, the exact inverse works on
// 64-bit numerators over L = lcm(n)^2 with a run-time division, and every
// table (quantiser classes, scales, inverse weights) comes from the kernel
// argument the host fills.
#include "codec_tile.hpp"
#include "settle.hpp"

namespace adct {
namespace {

// round-half-to-even(n / L) clipped to [0, 255] for a 64-bit numerator and a
// run-time L < 2^53: the float64 quotient of u = 2 clip(n) + L by 2L is off by
// at most one from floor(u / 2L), which the exact remainder corrects; a zero
// remainder is an exact half, which goes to the even neighbour.
__device__ __forceinline__ int rne_div_clip_rt(int64_t n, int64_t L, double inv_2L) {
    const int64_t nc = n < 0 ? 0 : (n > 255 * L ? 255 * L : n);
    const int64_t u = 2 * nc + L;
    const int64_t l2 = 2 * L;
    int q = int(double(u) * inv_2L);
    int64_t rem = u - int64_t(q) * l2;
    if (rem < 0) {
        --q;
        rem += l2;
    } else if (rem >= l2) {
        ++q;
        rem -= l2;
    }
    return q - int((rem == 0) & (q & 1));
}

// ---- exact near-half decisions (quantiser steps that admit exact halves)

// Pixel (x, y) of a dequantised block, rounded half to even exactly, given its
// float64 value v near the half fl + 1/2 (fl = floor(v)): the sign of
// D (2 pixel - 2 fl - 1) = 2 step sum_c N_c sqrt(r_c) - (2 fl + 1) D decides.
template <int BAND>
__device__ int settle_pixel(const RtMatArgs &m, const int (&C)[8][8], int step, int x, int y, double v) {
    constexpr int KB = BAND + 1 < 8 ? BAND + 1 : 8;
    int64_t n0 = 0, n1 = 0, n2 = 0, n3 = 0;
    for (int k = 0; k < KB; ++k)
        for (int l = 0; l < KB; ++l) {
            if (k + l > BAND) continue;
            const int64_t t = int64_t(C[k][l]) * (m.t[8 * k + x] * m.t[8 * l + y]) * m.st.w[8 * k + l];
            const int c = m.st.cls[8 * k + l];
            n0 += c == 0 ? t : 0;
            n1 += c == 1 ? t : 0;
            n2 += c == 2 ? t : 0;
            n3 += c == 3 ? t : 0;
        }
    const int64_t fl = int64_t(floor(v));
    const i128 g = m.st.g, s2 = 2 * i128(step);
    const i128 a = g * (s2 * n0 - i128(2 * fl + 1) * m.st.D);
    const int s = sgn_field(a, g * s2 * n1, g * s2 * n2, s2 * n3, uint32_t(m.st.p), uint32_t(m.st.q));
    return int(s > 0 ? fl + 1 : s < 0 ? fl : fl + (fl & 1));
}

// FIN: the decoder reads float32 B (coef_f) instead of integer coefficients.
template <int BAND, bool QUANT, int MODE, bool FIN>
__device__ __forceinline__ void process_tile_rt(const CodecArgs &a, const RtMatArgs &m,
                                                const Tile &t, const uint32_t (&pix)[8][2]) {
    constexpr int KB = BAND + 1 < 8 ? BAND + 1 : 8;
    constexpr int NZ = (BAND >= 14) ? 64 : (BAND + 1) * (BAND + 2) / 2;
    const PlaneArg &P = a.pl[t.p];
    const bool active = t.active;
    const int64_t gblk = int64_t(t.f) * a.blocks_per_frame + P.block_off + t.b;

    int C[8][8];       // what the integer decoder sees: Y (zonal) or q (quantised)
    double Bd[8][8];   // float decode: B as read
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            C[k][l] = 0;
            Bd[k][l] = 0.0;
        }

    if constexpr (MODE != kDecode) {
        // row pass Z[x][l] = sum_j T[l][j] A[x][j], then column pass
        // Y[k][l] = sum_x T[k][x] Z[x][l], inside the band only
        int Z[8][KB];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int xin[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) xin[j] = byte_of(pix[x][j >> 2], j & 3);
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                int acc = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) acc += m.t[8 * l + j] * xin[j];
                Z[x][l] = acc;
            }
        }
        int Y[8][8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                if (k + l > BAND) continue;
                int acc = 0;
#pragma unroll
                for (int x = 0; x < 8; ++x) acc += m.t[8 * k + x] * Z[x][l];
                Y[k][l] = acc;
            }
#pragma unroll
        for (int z = 0; z < NZ; ++z) {
            const int k = kZZ[z] >> 3, l = kZZ[z] & 7;
            int v = Y[k][l];
            if constexpr (QUANT) {
                const int mu = m.mu[8 * k + l];
                v = mu ? quant_rational(v, a.step, mu, m.inv_2mu[8 * k + l], a.inv_step_f)
                       : quant_irrational(v, m.skl[8 * k + l], a.inv_step_d);
            }
            C[k][l] = (z < a.r) ? v : 0;
        }
        if (active && a.coef) {
            int16_t *dst = a.coef + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r) dst[z] = int16_t(C[kZZ[z] >> 3][kZZ[z] & 7]);
        }
        if (active && a.coef_f) {
            float *dst = a.coef_f + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r) {
                    const int k = kZZ[z] >> 3, l = kZZ[z] & 7;
                    dst[z] = float(Y[k][l]) * float(m.skl[8 * k + l]);
                }
        }
    } else if (active) {
        if constexpr (FIN) {
            const float *src = a.coef_f + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r) Bd[kZZ[z] >> 3][kZZ[z] & 7] = double(src[z]);
        } else {
            const int16_t *src = a.coef + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r) C[kZZ[z] >> 3][kZZ[z] & 7] = src[z];
        }
    }

    if constexpr (MODE == kEncode) return;

    uint8_t *dst = a.out ? a.out + int64_t(t.f) * a.fs_out + P.out_off + t.out_off : nullptr;
    uint32_t sq = 0, cross = 0;
    if constexpr (!QUANT && !FIN) {
        // exact: A L = T^T (Y o c c^T) T, one output row x at a time:
        // U[l] = sum_k T[k][x] c_k c_l Y[k][l], pixel (x, y) = sum_l T[l][y] U[l]
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int64_t U[KB];
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                int64_t acc = 0;
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    if (k + l > BAND) continue;
                    acc += int64_t(m.t[8 * k + x]) * (int64_t(C[k][l]) * m.ckl[8 * k + l]);
                }
                U[l] = acc;
            }
            int q[8];
#pragma unroll
            for (int y = 0; y < 8; ++y) {
                int64_t acc = 0;
#pragma unroll
                for (int l = 0; l < KB; ++l) acc += int64_t(m.t[8 * l + y]) * U[l];
                q[y] = rne_div_clip_rt(acc, m.L, m.inv_2L);
            }
            const u32x2 v = emit_row(q, MODE == kEvaluate ? pix[x][0] : 0u,
                                     MODE == kEvaluate ? pix[x][1] : 0u, sq, cross);
            if (active && dst) __builtin_nontemporal_store(v, (u32x2 *)(dst + x * P.pitch_out));
        }
    } else {
        // float64: A = C_hat^T B' C_hat with B' = step q (quantised) or the B read,
        // C_hat = S T, so B'_kl s_k s_l enters the integer matrix products
        // near-half tolerance of the block: the float64 error bound
        // tol_c sum |C_kl| s_k s_l, at least 1e-6
        double tol = 1e-6;
        if (QUANT && !FIN && m.st.on) {
            double sc = 0.0;
#pragma unroll
            for (int k = 0; k < KB; ++k)
#pragma unroll
                for (int l = 0; l < KB; ++l)
                    if (k + l <= BAND) sc += fabs(double(C[k][l])) * m.skl[8 * k + l];
            tol = fmax(tol, sc * m.st.tol_c);
        }
        double W[KB][KB];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                if (k + l > BAND) {
                    W[k][l] = 0.0;
                    continue;
                }
                const double b = FIN ? Bd[k][l] : double(C[k][l]) * a.step_d;
                W[k][l] = b * m.skl[8 * k + l];
            }
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            double U[KB];
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    if (k + l > BAND) continue;
                    acc = fma(double(m.t[8 * k + x]), W[k][l], acc);
                }
                U[l] = acc;
            }
            int q[8];
#pragma unroll
            for (int y = 0; y < 8; ++y) {
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < KB; ++l) acc = fma(double(m.t[8 * l + y]), U[l], acc);
                q[y] = clamp255(rne_i32(acc));
                if (QUANT && !FIN && m.st.on) {
                    const double h = floor(acc) + 0.5;
                    if (fabs(acc - h) < tol && acc > -1.0 && acc < 256.0)
                        q[y] = clamp255(settle_pixel<BAND>(m, C, a.step, x, y, acc));
                }
            }
            const u32x2 v = emit_row(q, MODE == kEvaluate ? pix[x][0] : 0u,
                                     MODE == kEvaluate ? pix[x][1] : 0u, sq, cross);
            if (active && dst) __builtin_nontemporal_store(v, (u32x2 *)(dst + x * P.pitch_out));
        }
    }

    if constexpr (MODE == kEvaluate) {
        unsigned e = active ? sq - 2u * cross : 0u;
        e = wave_sum(e);
        if ((threadIdx.x & 63) == 0 && e)
            atomicAdd(a.sse + int64_t(t.f) * a.n_planes + t.p, (unsigned long long)e);
    }
}

// One 64-block tile per wave and no persistent loop: the kernel is straight-line
// code, so the table values it reads from its argument are loaded where they
// are needed rather than kept live across iterations.
template <int BAND, bool QUANT, int MODE, bool FIN>
__global__ __launch_bounds__(256) void k_codec_rt(const CodecArgs a, const RtMatArgs m) {
    const int lane = threadIdx.x & 63;
    const int total = a.n_frames * a.waves_per_frame;
    const int gw = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    if (gw >= total) return;
    uint32_t pix[8][2];
    const Tile t = tile_of(a, gw, lane);
    if constexpr (MODE != kDecode) load_tile(a, t, pix);
    process_tile_rt<BAND, QUANT, MODE, FIN>(a, m, t, pix);
}

template <int BAND, bool QUANT, int MODE, bool FIN>
adct_status launch_rt_one(const CodecArgs &a, const RtMatArgs &m, int total_waves, hipStream_t s) {
    const int64_t grid = (int64_t(total_waves) + 3) / 4;
    hipLaunchKernelGGL((k_codec_rt<BAND, QUANT, MODE, FIN>), dim3(unsigned(grid)), dim3(256), 0, s, a, m);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

template <int BAND>
adct_status launch_rt_band(bool quant, bool float_in, Mode mode, const CodecArgs &a,
                           const RtMatArgs &m, int tw, hipStream_t s) {
    if (mode == kDecode && float_in) return launch_rt_one<BAND, false, kDecode, true>(a, m, tw, s);
    if (quant) {
        if (mode == kEncode) return launch_rt_one<BAND, true, kEncode, false>(a, m, tw, s);
        if (mode == kDecode) return launch_rt_one<BAND, true, kDecode, false>(a, m, tw, s);
        return launch_rt_one<BAND, true, kEvaluate, false>(a, m, tw, s);
    }
    if (mode == kEncode) return launch_rt_one<BAND, false, kEncode, false>(a, m, tw, s);
    if (mode == kDecode) return launch_rt_one<BAND, false, kDecode, false>(a, m, tw, s);
    return launch_rt_one<BAND, false, kEvaluate, false>(a, m, tw, s);
}

}  // namespace

adct_status launch_codec_rt(int band, bool quant, bool float_in, Mode mode, const CodecArgs &a,
                            const RtMatArgs &m, int total_waves, hipStream_t s) {
    if (total_waves <= 0) return ADCT_OK;
    if (band <= 3) return launch_rt_band<3>(quant, float_in, mode, a, m, total_waves, s);
    return launch_rt_band<14>(quant, float_in, mode, a, m, total_waves, s);
}

}  // namespace adct
