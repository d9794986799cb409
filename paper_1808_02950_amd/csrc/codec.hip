// Fused blockwise 8x8 transform coding on gfx950 (Sec. 6.1.1 of the paper):
// forward T A T^T -> scale / zonal zig-zag (-> quantiser) -> inverse -> round,
// clip -> squared error.  One lane owns one 8x8 block for the whole pipeline,
// so both 1-D passes and the transpose between them stay in registers; a
// wave covers 64 consecutive blocks of a plane in raster order and every row
// load / store of the wave is one contiguous 512-byte run.
#include <algorithm>
#include <type_traits>

#include "codec_tile.hpp"

namespace adct {
namespace {

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

// acc + c v for a small constant c (0, +-1, +-2); float64 uses one fma.
template <class V>
__device__ __forceinline__ V mac(V acc, V v, int c) {
    if constexpr (std::is_same<V, double>::value) {
        if (c == 1) return acc + v;
        if (c == -1) return acc - v;
        return fma(v, double(c), acc);
    } else {
        if (c == 1) return acc + v;
        if (c == -1) return acc - v;
        if (c == 2) return acc + (v + v);
        return acc - (v + v);
    }
}

template <class V>
__device__ __forceinline__ V cmul(V v, int c) {
    if (c == 1) return v;
    if (c == -1) return -v;
    return v * V(c);
}

// Inverse 8-point transform x = T^T y when only y[0..K) can be nonzero:
// x_m = e_m + o_m, x_{7-m} = e_m - o_m with e from the even rows, o from the odd.
template <int ID, int K, class V>
__device__ __forceinline__ void inv8(const V (&y)[8], V (&x)[8], int kmax = K - 1) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        V e = V(0), o = V(0);
        bool he = false, ho = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int c = Tf<ID>::t(k, m);
            if (c == 0 || k > kmax) continue;
            if (k & 1) {
                o = ho ? mac(o, y[k], c) : cmul(y[k], c);
                ho = true;
            } else {
                e = he ? mac(e, y[k], c) : cmul(y[k], c);
                he = true;
            }
        }
        if (he && ho) {
            x[m] = e + o;
            x[7 - m] = e - o;
        } else if (he) {
            x[m] = e;
            x[7 - m] = e;
        } else if (ho) {
            x[m] = o;
            x[7 - m] = -o;
        } else {
            x[m] = V(0);
            x[7 - m] = V(0);
        }
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

// ------------------------------------------------------------------ kernel
//
// BAND: only coefficients (k, l) with k + l <= BAND can be retained (r <= 10
// needs BAND 3; 14 is the whole block).  The retained set inside the band is
// the zig-zag prefix of length r (runtime).
//
// The grid is persistent: each wave walks tiles gw, gw + stride, ... (a tile is
// 64 consecutive blocks of one plane of one frame) and issues the loads of its
// next tile before it transforms the current one.

// Store the r retained coefficients C of the lane's block (zig-zag order) at
// coef[gblk * r ...].  A full tile's coefficients are one contiguous run of
// 128 r bytes: for even r whose dword stride r/2 is not a multiple of 4 (so
// the LDS writes are free of bank conflicts beyond two-way) and a 16-byte
// aligned run, they go through a per-wave LDS slice and leave as 16-byte
// stores that cover whole lines, instead of r/2 scattered 4-byte stores a lane.
template <int NZ>
__device__ __forceinline__ void store_coef_tile(const CodecArgs &a, const Tile &t, const PlaneArg &P,
                                                int64_t gblk, const int (&C)[8][8]) {
    if (!a.coef) return;
    const int lane = int(threadIdx.x & 63);
    const int64_t run0 = (gblk - lane) * a.r;           // first int16 of the tile
    const bool staged = (a.r & 1) == 0 && ((a.r >> 1) & 3) != 0 && t.b - lane + 64 <= P.nblocks &&
                        ((reinterpret_cast<uintptr_t>(a.coef + run0) & 15) == 0);
    if (staged) {
        __shared__ uint32_t stage[4][NZ * 32];
        uint32_t *slice = stage[threadIdx.x >> 6];
        const int half_r = a.r >> 1;
#pragma unroll
        for (int z = 0; z < NZ; z += 2) {
            if (z + 1 < a.r) {
                const int k0 = kZZ[z] >> 3, l0 = kZZ[z] & 7;
                const int k1 = kZZ[z + 1] >> 3, l1 = kZZ[z + 1] & 7;
                slice[lane * half_r + (z >> 1)] =
                    (uint32_t(C[k0][l0]) & 0xffffu) | (uint32_t(C[k1][l1]) << 16);
            }
        }
        __builtin_amdgcn_wave_barrier();
        const int chunks = 8 * a.r;                      // 16-byte pieces of the run
        u32x4 *gdst = reinterpret_cast<u32x4 *>(a.coef + run0);
        for (int c = lane; c < chunks; c += 64)
            __builtin_nontemporal_store(reinterpret_cast<const u32x4 *>(slice)[c], gdst + c);
        __builtin_amdgcn_wave_barrier();
        return;
    }
    if (!t.active) return;
    int16_t *dst = a.coef + gblk * a.r;
    if (a.r == NZ && (NZ & 1) == 0) {             // whole band, no per-entry test
#pragma unroll
        for (int z = 0; z < NZ; z += 2) {
            const int k0 = kZZ[z] >> 3, l0 = kZZ[z] & 7;
            const int k1 = kZZ[z + 1] >> 3, l1 = kZZ[z + 1] & 7;
            const uint32_t pk = (uint32_t(C[k0][l0]) & 0xffffu) | (uint32_t(C[k1][l1]) << 16);
            __builtin_nontemporal_store(pk, (uint32_t *)(dst + z));
        }
    } else if ((a.r & 1) == 0) {
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

// The bandwidth probe: the loads and stores of an evaluation with no
// arithmetic.  The reconstruction receives the input pixels, the coefficients
// receive bytes of them.
template <int BAND>
__device__ __forceinline__ void probe_tile(const CodecArgs &a, const Tile &t, const uint32_t (&pix)[8][2]) {
    constexpr int NZ = (BAND >= 14) ? 64 : (BAND + 1) * (BAND + 2) / 2;
    const PlaneArg &P = a.pl[t.p];
    const int64_t gblk = int64_t(t.f) * a.blocks_per_frame + P.block_off + t.b;
    int C[8][8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int l = 0; l < 8; ++l) C[k][l] = int(pix[(8 * k + l) & 7][((8 * k + l) >> 3) & 1] >> (l & 1 ? 16 : 0));
    store_coef_tile<NZ>(a, t, P, gblk, C);
    uint8_t *dst = a.out ? a.out + int64_t(t.f) * a.fs_out + P.out_off + t.out_off : nullptr;
    if (t.active && dst) {
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            u32x2 v;
            v.x = pix[x][0];
            v.y = pix[x][1];
            __builtin_nontemporal_store(v, (u32x2 *)(dst + x * P.pitch_out));
        }
    }
}

template <int ID, int BAND, bool QUANT, int MODE>
__device__ __forceinline__ void process_tile(const CodecArgs &a, const QuantTables &qt, const Tile &t,
                                             const uint32_t (&pix)[8][2]) {
    if constexpr (MODE == kProbe) {
        probe_tile<BAND>(a, t, pix);
        return;
    }
    constexpr int KB = BAND + 1 < 8 ? BAND + 1 : 8;  // rows / columns touched
    const PlaneArg &P = a.pl[t.p];
    const bool active = t.active;
    const int64_t gblk = int64_t(t.f) * a.blocks_per_frame + P.block_off + t.b;

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
                if (Tf<ID>::mu(k, l) != 0)
                    v = quant_rational_f(v, qt.qc1[Tf<ID>::cls(k, l)], qt.qc2[Tf<ID>::cls(k, l)]);
                else
                    v = rne_i32(double(v) * qt.qinv[Tf<ID>::cls(k, l)]);   // never a half: see quant_irrational
            }
            C[k][l] = (z < a.r) ? v : 0;
        }
        store_coef_tile<NZ>(a, t, P, gblk, C);
        if (active && a.coef_f) {
            float *dst = a.coef_f + gblk * a.r;
#pragma unroll
            for (int z = 0; z < NZ; ++z)
                if (z < a.r)
                    dst[z] = float(Y[kZZ[z] >> 3][kZZ[z] & 7]) *
                             float(Tf<ID>::skl(kZZ[z] >> 3, kZZ[z] & 7));
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
    uint8_t *dst = a.out ? a.out + int64_t(t.f) * a.fs_out + P.out_off + t.out_off : nullptr;
    uint32_t sq = 0, cross = 0;
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
            inv8<ID, KB>(yin, xo, BAND - l);
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
            const u32x2 v = emit_row(q, MODE == kEvaluate ? pix[x][0] : 0u,
                                     MODE == kEvaluate ? pix[x][1] : 0u, sq, cross);
            if (active && dst) __builtin_nontemporal_store(v, (u32x2 *)(dst + x * P.pitch_out));
        }
    } else {
        // dequantised B = step q, A = C_hat^T B C_hat in float64.  The column
        // pass runs over row pairs (x, 7 - x): row k of T is symmetric for even
        // k and antisymmetric for odd k, so U[x][l] = e + o and
        // U[7 - x][l] = e - o with e, o the even- and odd-k sums.  Only two rows
        // of the intermediate are live at a time.
        double Yd[KB][KB];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int l = 0; l < KB; ++l)
                // q step is exact in float64 (|q| < 2^15, step < 2^16) and needs no
                // quarter-rate 32-bit integer multiply
                Yd[k][l] = (k + l <= BAND) ? double(C[k][l]) * qt.qdeq[Tf<ID>::cls(k, l)] : 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            double yin0[8], yin1[8];
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                yin0[l] = 0.0;
                yin1[l] = 0.0;
            }
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                double e = 0.0, o = 0.0;
                bool he = false, ho = false;
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    if (k + l > BAND) continue;
                    const int tk = Tf<ID>::t(k, x);
                    if (tk == 0) continue;
                    const double v = Yd[k][l];
                    if (k & 1) {
                        o = ho ? fma(double(tk), v, o) : double(tk) * v;
                        ho = true;
                    } else {
                        e = he ? fma(double(tk), v, e) : double(tk) * v;
                        he = true;
                    }
                }
                yin0[l] = ho ? e + o : e;
                yin1[l] = ho ? e - o : e;
            }
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int xr = half ? 7 - x : x;
                double xo[8];
                inv8<ID, KB>(half ? yin1 : yin0, xo);
                int q[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) q[m] = rne_i32(xo[m]);
                const u32x2 v = emit_row_sat(q, MODE == kEvaluate ? pix[xr][0] : 0u,
                                             MODE == kEvaluate ? pix[xr][1] : 0u, sq, cross);
                if (active && dst) __builtin_nontemporal_store(v, (u32x2 *)(dst + xr * P.pitch_out));
            }
        }
    }

    if constexpr (MODE == kEvaluate) {
        unsigned e = active ? sq - 2u * cross : 0u;
        e = wave_sum(e);
        if ((threadIdx.x & 63) == 0 && e)
            atomicAdd(a.sse + int64_t(t.f) * a.n_planes + t.p, (unsigned long long)e);
    }
}

template <int ID, int BAND, bool QUANT, int MODE>
__global__ __launch_bounds__(256) void k_codec(const CodecArgs a, const QuantTables qt) {
    const int lane = threadIdx.x & 63;
    const int total = a.n_frames * a.waves_per_frame;
    const int stride = int(gridDim.x) * 4;
    int gw = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    if (gw >= total) return;                               // whole wave leaves
    // two pixel buffers used in turn: the next tile loads into one while the
    // current tile is transformed from the other.  The next loads are issued
    // on every pass (a wave's last pass re-reads its current tile), so no
    // branch joins paths with different loads in flight and the waits for the
    // current tile leave the next tile's loads outstanding.
    uint32_t pa[8][2], pb[8][2];
    Tile ta = tile_of(a, gw, lane), tb = ta;
    if constexpr (MODE != kDecode) load_tile(a, ta, pa);
    while (true) {
        int nxt = gw + stride;
        bool more = nxt < total;                           // wave-uniform
        tb = tile_of(a, more ? nxt : gw, lane);
        if constexpr (MODE != kDecode) load_tile(a, tb, pb);
        process_tile<ID, BAND, QUANT, MODE>(a, qt, ta, pa);
        if (!more) break;
        gw = nxt;
        nxt = gw + stride;
        more = nxt < total;
        ta = tile_of(a, more ? nxt : gw, lane);
        if constexpr (MODE != kDecode) load_tile(a, ta, pa);
        process_tile<ID, BAND, QUANT, MODE>(a, qt, tb, pb);
        if (!more) break;
        gw = nxt;
    }
}


template <int ID, int BAND, bool QUANT, int M>
adct_status launch_one(const CodecArgs &a, const QuantTables &q, int total_waves, hipStream_t s) {
    auto kern = k_codec<ID, BAND, QUANT, M>;
    int grid = 0;
    adct_status st = persistent_grid(kern, total_waves, &grid);
    if (st) return st;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, a, q);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

template <int ID, int BAND, bool QUANT>
adct_status launch_mode(Mode mode, const CodecArgs &a, const QuantTables &q, int total_waves, hipStream_t s) {
    if (mode == kEncode) return launch_one<ID, BAND, QUANT, kEncode>(a, q, total_waves, s);
    if (mode == kDecode) return launch_one<ID, BAND, QUANT, kDecode>(a, q, total_waves, s);
    return launch_one<ID, BAND, QUANT, kEvaluate>(a, q, total_waves, s);
}

template <int ID>
adct_status launch_tf(int band, bool quant, Mode mode, const CodecArgs &a, const QuantTables &q, int tw, hipStream_t s) {
    if (band <= 3) return quant ? launch_mode<ID, 3, true>(mode, a, q, tw, s) : launch_mode<ID, 3, false>(mode, a, q, tw, s);
    return quant ? launch_mode<ID, 14, true>(mode, a, q, tw, s) : launch_mode<ID, 14, false>(mode, a, q, tw, s);
}

}  // namespace

adct_status launch_codec(int tid, int band, bool quant, Mode mode, const CodecArgs &a,
                         const QuantTables &q, int total_waves, hipStream_t s) {
    if (total_waves <= 0) return ADCT_OK;
    if (mode == kProbe)
        return band <= 3 ? launch_one<ADCT_T1, 3, false, kProbe>(a, q, total_waves, s)
                         : launch_one<ADCT_T1, 14, false, kProbe>(a, q, total_waves, s);
    switch (tid) {
        case ADCT_T1: return launch_tf<ADCT_T1>(band, quant, mode, a, q, total_waves, s);
        case ADCT_T2: return launch_tf<ADCT_T2>(band, quant, mode, a, q, total_waves, s);
        case ADCT_LO: return launch_tf<ADCT_LO>(band, quant, mode, a, q, total_waves, s);
        case ADCT_T6: return launch_tf<ADCT_T6>(band, quant, mode, a, q, total_waves, s);
        case ADCT_RDCT: return launch_tf<ADCT_RDCT>(band, quant, mode, a, q, total_waves, s);
        case ADCT_T4: return launch_tf<ADCT_T4>(band, quant, mode, a, q, total_waves, s);
        default: return fail(ADCT_ENOTSUP, "transform not implemented by the integer codec");
    }
}

}  // namespace adct
