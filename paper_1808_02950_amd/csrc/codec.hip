// Fused blockwise 8x8 transform coding on gfx950 (Sec. 6.1.1 of the paper):
// forward T A T^T -> scale / zonal zig-zag (-> quantiser) -> inverse -> round,
// clip -> squared error.  One lane owns one 8x8 block for the whole pipeline,
// so both 1-D passes and the transpose between them stay in registers; a
// wave covers 64 consecutive blocks of a plane in raster order and every row
// load / store of the wave is one contiguous 512-byte run.
#include "adct_internal.hpp"

namespace adct {
namespace {

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ 1-D passes

// Forward 8-point transform y = T x for the outputs y[0..NOUT).  T1 uses the
// paper's fast algorithm T1 = D A4 A3 A2 A1 (Sec. 5.1): 24 additions and 6
// doublings; the other matrices use the even/odd butterfly their symmetry
// allows (one stage of 8 additions, then 4x4 products with entries 0, +-1, +-2).
template <int ID, int NOUT, class V>
__device__ __forceinline__ void fwd8(const V (&x)[8], V (&y)[8]) {
    if constexpr (ID == ADCT_T1) {
        const V a0 = x[0] + x[7], a1 = x[1] + x[6], a2 = x[2] + x[5], a3 = x[3] + x[4];
        const V a4 = x[3] - x[4], a5 = x[2] - x[5], a6 = x[1] - x[6], a7 = x[0] - x[7];
        const V b0 = a0 + a3, b1 = a1 + a2, b2 = a1 - a2, b3 = a0 - a3;
        y[0] = b0 + b1;
        y[4] = b0 - b1;
        y[2] = b2 + (b3 + b3);
        y[6] = b3 - (b2 + b2);
        const V a67 = a6 + a7, a45 = a4 + a5;
        y[1] = a5 + (a67 + a67);
        y[3] = a7 - (a45 + a45);
        const V a76 = a7 - a6, a54 = a5 - a4;
        y[5] = a4 + (a76 + a76);
        y[7] = (a54 + a54) - a6;
    } else {
        V s[4], d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            s[m] = x[m] + x[7 - m];
            d[m] = x[m] - x[7 - m];
        }
#pragma unroll
        for (int k = 0; k < NOUT; ++k) {
            V acc = V(0);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int c = Tf<ID>::t(k, m);
                const V v = (k & 1) ? d[m] : s[m];
                if (c == 1) acc = acc + v;
                else if (c == -1) acc = acc - v;
                else if (c == 2) acc = acc + (v + v);
                else if (c == -2) acc = acc - (v + v);
            }
            y[k] = acc;
        }
    }
}

// Inverse 8-point transform x = T^T y when only y[0..K) can be nonzero:
// x_m = e_m + o_m, x_{7-m} = e_m - o_m with e from the even rows, o from the odd.
template <int ID, int K, class V>
__device__ __forceinline__ void inv8(const V (&y)[8], V (&x)[8]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        V e = V(0), o = V(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int c = Tf<ID>::t(k, m);
            V &acc = (k & 1) ? o : e;
            if (c == 1) acc = acc + y[k];
            else if (c == -1) acc = acc - y[k];
            else if (c == 2) acc = acc + (y[k] + y[k]);
            else if (c == -2) acc = acc - (y[k] + y[k]);
        }
        x[m] = e + o;
        x[7 - m] = e - o;
    }
}

// ------------------------------------------------------------------ helpers

// round-half-to-even(n / L) clipped to [0, 255] for the exact inverse numerator
// n (|n| < 2^31).  Clipping first keeps 2n + L below 2^31.
template <int32_t L>
__device__ __forceinline__ int rne_div_clip(int n) {
    const int nc = min(max(n, 0), 255 * L);
    const uint32_t u = 2u * uint32_t(nc) + uint32_t(L);          // < 511 L
    const uint32_t q = u / uint32_t(2 * L);                         // round half up
    const bool tie = (u == uint32_t(__umul24(q, uint32_t(2 * L))));
    return int(q) - int(tie & (q & 1u));
}

__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d) {
    return uint32_t(a) | (uint32_t(b) << 8) | (uint32_t(c) << 16) | (uint32_t(d) << 24);
}

__device__ __forceinline__ int byte_of(uint32_t w, int i) { return int((w >> (8 * i)) & 0xffu); }

// round-half-away(Y / d) for the rational classes: floor((2|Y| + d) / (2d)) with
// qden = 2d, exact for 2|Y| + d < 2^24 (float estimate, integer correction).
__device__ __forceinline__ int quant_rational(int y, int32_t qden, float qinv) {
    const int ay = y < 0 ? -y : y;
    const int num = 2 * ay + (qden >> 1);
    int q = int(float(num) * qinv);
    const int rem = num - __mul24(q, qden);
    q += (rem >= qden) ? 1 : 0;
    q -= (rem < 0) ? 1 : 0;
    return y < 0 ? -q : q;
}

// round-half-away(Y * alpha) for irrational classes (never an exact half; the
// nearest half is > 1e-9 away for |Y| < 2^16, far above the float64 error).
__device__ __forceinline__ int quant_irrational(int y, double alpha) {
    const double x = double(y < 0 ? -y : y) * alpha;
    const int q = int(floor(x + 0.5));
    return y < 0 ? -q : q;
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------ kernel
//
// BAND: only coefficients (k, l) with k + l <= BAND can be retained (r <= 10
// needs BAND 3; 14 is the whole block).  The retained set inside the band is
// the zig-zag prefix of length r (runtime).

template <int ID, int BAND, bool QUANT, int MODE>
__global__ __launch_bounds__(256) void k_codec(const CodecArgs a) {
    constexpr int KB = BAND + 1 < 8 ? BAND + 1 : 8;  // rows / columns touched
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gw >= a.n_frames * a.waves_per_frame) return;  // whole wave leaves
    const int f = gw / a.waves_per_frame;
    const int w = gw - f * a.waves_per_frame;
    int p = 0;
    while (p + 1 < a.n_planes && w >= a.pl[p + 1].wave_start) ++p;
    const PlaneArg P = a.pl[p];
    const int b = (w - P.wave_start) * 64 + lane;
    const bool active = b < P.nblocks;
    const int by = active ? b / P.nbx : 0;
    const int bx = active ? b - by * P.nbx : 0;
    const int64_t gblk = int64_t(f) * a.blocks_per_frame + P.block_off + b;

    // ---- pixels in (8 bytes per row) --------------------------------------
    uint32_t pix[8][2];
    if constexpr (MODE != kDecode) {
        const uint8_t *src = a.in + int64_t(f) * a.fs_in + P.in_off +
                             int64_t(8 * by) * P.pitch_in + 8 * bx;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            u32x2 v = {0u, 0u};
            if (active) v = __builtin_nontemporal_load((const u32x2 *)(src + int64_t(x) * P.pitch_in));
            pix[x][0] = v.x;
            pix[x][1] = v.y;
        }
    }

    // ---- coefficients inside the band --------------------------------------
    int Y[8][8];  // Y[k][l] (only k + l <= BAND meaningful)
    if constexpr (MODE != kDecode) {
        // row pass: Z[x][l] = sum_m T[l][m] A[x][m], l < KB
        int Z[8][8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int xin[8], yout[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int m = 0; m < 8; ++m) xin[m] = byte_of(pix[x][m >> 2], m & 3);
            fwd8<ID, KB>(xin, yout);
#pragma unroll
            for (int l = 0; l < 8; ++l) Z[x][l] = yout[l];
        }
        // column pass: Y[k][l] = sum_x T[k][x] Z[x][l]
#pragma unroll
        for (int l = 0; l < KB; ++l) {
            int cin[8], cout[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int x = 0; x < 8; ++x) cin[x] = Z[x][l];
            fwd8<ID, KB>(cin, cout);
#pragma unroll
            for (int k = 0; k < 8; ++k) Y[k][l] = cout[k];
        }
    }

    // ---- quantise / store / load coefficients ------------------------------
    constexpr int NZ = (BAND >= 14) ? 64 : (BAND + 1) * (BAND + 2) / 2;
    int C[8][8];  // what the decoder sees: Y (zonal) or q (quantised)
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int l = 0; l < 8; ++l) C[k][l] = 0;

    if constexpr (MODE != kDecode) {
#pragma unroll
        for (int z = 0; z < NZ; ++z) {
            const int k = kZZ[z] >> 3, l = kZZ[z] & 7;
            int v = Y[k][l];
            if constexpr (QUANT) {
                const int i = kZZ[z];
                v = a.qden[i] ? quant_rational(v, a.qden[i], a.qinv[i])
                              : quant_irrational(v, a.qalpha[i]);
            }
            C[k][l] = (z < a.r) ? v : 0;
        }
        if (active && a.coef) {
            int16_t *dst = a.coef + gblk * a.r;
            if ((a.r & 1) == 0) {
#pragma unroll
                for (int z = 0; z < NZ; z += 2) {
                    if (z + 1 < a.r) {
                        const int k0 = kZZ[z] >> 3, l0 = kZZ[z] & 7;
                        const int k1 = kZZ[z + 1] >> 3, l1 = kZZ[z + 1] & 7;
                        const uint32_t pk = (uint32_t(C[k0][l0]) & 0xffffu) | (uint32_t(C[k1][l1]) << 16);
                        __builtin_nontemporal_store(pk, (uint32_t *)(dst + z));
                    }
                }
            } else {
#pragma unroll
                for (int z = 0; z < NZ; ++z)
                    if (z < a.r) dst[z] = int16_t(C[kZZ[z] >> 3][kZZ[z] & 7]);
            }
        }
        if (active && a.coef_f) {
            float *dst = a.coef_f + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r) dst[z] = float(Y[kZZ[z] >> 3][kZZ[z] & 7]) * a.bscale[kZZ[z]];
        }
    } else {
        if (active) {
            const int16_t *srcc = a.coef + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r) C[kZZ[z] >> 3][kZZ[z] & 7] = srcc[z];
        }
    }

    if constexpr (MODE == kEncode) return;

    // ---- inverse, round, clip, store, squared error ------------------------
    uint8_t *dst = a.out ? a.out + int64_t(f) * a.fs_out + P.out_off +
                               int64_t(8 * by) * P.pitch_out + 8 * bx
                         : nullptr;
    unsigned err = 0;
    if constexpr (!QUANT) {
        // exact: A L = T^T (Y o c c^T) T with c_k = L1 / n_k, L = L1^2
        constexpr int32_t L = Tf<ID>::L();
        int U[8][8];  // U[x][l] = sum_k T[k][x] c_k Y[k][l] c_l
#pragma unroll
        for (int l = 0; l < KB; ++l) {
            int yin[8], xo[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                yin[k] = (k < KB) ? __mul24(C[k][l], Tf<ID>::c(k) * Tf<ID>::c(l)) : 0;
            inv8<ID, KB>(yin, xo);
#pragma unroll
            for (int x = 0; x < 8; ++x) U[x][l] = xo[x];
        }
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int yin[8], xo[8];
#pragma unroll
            for (int l = 0; l < 8; ++l) yin[l] = (l < KB) ? U[x][l] : 0;
            inv8<ID, KB>(yin, xo);
            int q[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) q[m] = rne_div_clip<L>(xo[m]);
            if constexpr (MODE == kEvaluate) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int d = q[m] - byte_of(pix[x][m >> 2], m & 3);
                    err += unsigned(__mul24(d, d));
                }
            }
            if (active && dst) {
                const u32x2 v = {pack4(q[0], q[1], q[2], q[3]), pack4(q[4], q[5], q[6], q[7])};
                __builtin_nontemporal_store(v, (u32x2 *)(dst + int64_t(x) * P.pitch_out));
            }
        }
    } else {
        // dequantised B = step q, A = C_hat^T B C_hat in float64
        double U[8][8];
#pragma unroll
        for (int l = 0; l < KB; ++l) {
            double yin[8], xo[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                yin[k] = (k < KB) ? double(C[k][l]) * a.dq[8 * k + l] : 0.0;
            inv8<ID, KB>(yin, xo);
#pragma unroll
            for (int x = 0; x < 8; ++x) U[x][l] = xo[x];
        }
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            double yin[8], xo[8];
#pragma unroll
            for (int l = 0; l < 8; ++l) yin[l] = (l < KB) ? U[x][l] : 0.0;
            inv8<ID, KB>(yin, xo);
            int q[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) q[m] = int(fmin(fmax(rint(xo[m]), 0.0), 255.0));
            if constexpr (MODE == kEvaluate) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int d = q[m] - byte_of(pix[x][m >> 2], m & 3);
                    err += unsigned(__mul24(d, d));
                }
            }
            if (active && dst) {
                const u32x2 v = {pack4(q[0], q[1], q[2], q[3]), pack4(q[4], q[5], q[6], q[7])};
                __builtin_nontemporal_store(v, (u32x2 *)(dst + int64_t(x) * P.pitch_out));
            }
        }
    }

    if constexpr (MODE == kEvaluate) {
        if (!active) err = 0;
        err = wave_sum(err);
        if (lane == 0 && err) atomicAdd(a.sse + int64_t(f) * a.n_planes + p, (unsigned long long)err);
    }
}

template <int ID, int BAND, bool QUANT>
adct_status launch_mode(Mode mode, const CodecArgs &a, int total_waves, hipStream_t s) {
    const dim3 grid((total_waves + 3) / 4), block(256);
    if (mode == kEncode) hipLaunchKernelGGL((k_codec<ID, BAND, QUANT, kEncode>), grid, block, 0, s, a);
    else if (mode == kDecode) hipLaunchKernelGGL((k_codec<ID, BAND, QUANT, kDecode>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_codec<ID, BAND, QUANT, kEvaluate>), grid, block, 0, s, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

template <int ID>
adct_status launch_tf(int band, bool quant, Mode mode, const CodecArgs &a, int tw, hipStream_t s) {
    if (band <= 3) return quant ? launch_mode<ID, 3, true>(mode, a, tw, s) : launch_mode<ID, 3, false>(mode, a, tw, s);
    return quant ? launch_mode<ID, 14, true>(mode, a, tw, s) : launch_mode<ID, 14, false>(mode, a, tw, s);
}

}  // namespace

adct_status launch_codec(int tid, int band, bool quant, Mode mode, const CodecArgs &a,
                         int total_waves, hipStream_t s) {
    if (total_waves <= 0) return ADCT_OK;
    switch (tid) {
        case ADCT_T1: return launch_tf<ADCT_T1>(band, quant, mode, a, total_waves, s);
        case ADCT_T2: return launch_tf<ADCT_T2>(band, quant, mode, a, total_waves, s);
        case ADCT_LO: return launch_tf<ADCT_LO>(band, quant, mode, a, total_waves, s);
        case ADCT_T6: return launch_tf<ADCT_T6>(band, quant, mode, a, total_waves, s);
        case ADCT_RDCT: return launch_tf<ADCT_RDCT>(band, quant, mode, a, total_waves, s);
        case ADCT_T4: return launch_tf<ADCT_T4>(band, quant, mode, a, total_waves, s);
        default: return fail(ADCT_ENOTSUP, "transform not implemented by the integer codec");
    }
}

}  // namespace adct
