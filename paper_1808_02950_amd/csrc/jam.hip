// Blockwise N x N transform coding with the 16- and 32-point matrices that the
// Jridi-Alfalou-Meher construction grows from T1 (Sec. 6.2), on gfx950:
// forward T A T^T -> zonal zig-zag prefix (-> quantiser) -> inverse -> round,
// clip -> squared error, one pass over the pixels.
//
// The construction gives the N-point transform a butterfly form: output 2i is
// output i of the N/2-point transform of x_top + rev(x_bottom), output 2i + 1 the
// same of x_top - rev(x_bottom); the 8-point core is the paper's signal-flow
// graph of T1 (Sec. 5.1).  The inverse T^T runs the same graph backwards.
//
// Mapping: a wave owns 64/N horizontally adjacent blocks (a tile) and each lane
// one row of one block.  The lane loads its row, transforms it, and the rows go
// through LDS so that each lane then owns one column for the column transform,
// the quantiser and the column inverse; a second LDS pass returns the rows for
// the row inverse, rounding, the store and the squared error.  Only the columns
// 0..band (band = the last zig-zag diagonal the prefix reaches) go through LDS.
// A workgroup is one wave, so its barriers cost nothing and waves never wait on
// each other; the grid strides over the tiles.
#include <string.h>

#include <algorithm>

#include "adct_internal.hpp"
#include "wave.hpp"

namespace adct {
namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ transforms

// y = T1 x by the signal-flow graph of Sec. 5.1 (24 additions, 6 doublings).
template <class V>
__device__ __forceinline__ void t1_fwd(const V *x, V *y) {
    const V a0 = x[0] + x[7], a1 = x[1] + x[6], a2 = x[2] + x[5], a3 = x[3] + x[4];
    const V a4 = x[3] - x[4], a5 = x[2] - x[5], a6 = x[1] - x[6], a7 = x[0] - x[7];
    const V b0 = a0 + a3, b1 = a1 + a2, b2 = a1 - a2, b3 = a0 - a3;
    y[0] = b0 + b1;
    y[4] = b0 - b1;
    y[2] = b2 + (b3 + b3);
    y[6] = b3 - (b2 + b2);
    const V a67 = a6 + a7, a45 = a4 + a5, a76 = a7 - a6, a54 = a5 - a4;
    y[1] = a5 + (a67 + a67);
    y[3] = a7 - (a45 + a45);
    y[5] = a4 + (a76 + a76);
    y[7] = (a54 + a54) - a6;
}

// x = T1^T y: the same graph with every edge reversed.
template <class V>
__device__ __forceinline__ void t1_inv(const V *y, V *x) {
    const V b0 = y[0] + y[4], b1 = y[0] - y[4];
    const V b2 = y[2] - (y[6] + y[6]), b3 = (y[2] + y[2]) + y[6];
    const V y33 = y[3] + y[3], y77 = y[7] + y[7], y11 = y[1] + y[1], y55 = y[5] + y[5];
    const V a4 = (y[5] - y33) - y77;
    const V a5 = (y[1] - y33) + y77;
    const V a6 = (y11 - y55) - y[7];
    const V a7 = (y11 + y[3]) + y55;
    const V a0 = b0 + b3, a3 = b0 - b3, a1 = b1 + b2, a2 = b1 - b2;
    x[0] = a0 + a7;
    x[7] = a0 - a7;
    x[1] = a1 + a6;
    x[6] = a1 - a6;
    x[2] = a2 + a5;
    x[5] = a2 - a5;
    x[3] = a3 + a4;
    x[4] = a3 - a4;
}

// y = T_(N) x (rows in the sign convention of the printed matrices).
template <int N, class V>
__device__ __forceinline__ void jam_fwd(const V *x, V *y) {
    if constexpr (N == 8) {
        t1_fwd(x, y);
    } else {
        constexpr int H = N / 2;
        V s[H], d[H], ys[H], yd[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            s[i] = x[i] + x[N - 1 - i];
            d[i] = x[i] - x[N - 1 - i];
        }
        jam_fwd<H>(s, ys);
        jam_fwd<H>(d, yd);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            y[2 * i] = ys[i];
            y[2 * i + 1] = yd[i];
        }
    }
}

// x = T_(N)^T y.
template <int N, class V>
__device__ __forceinline__ void jam_inv(const V *y, V *x) {
    if constexpr (N == 8) {
        t1_inv(y, x);
    } else {
        constexpr int H = N / 2;
        V ye[H], yo[H], u[H], v[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            ye[i] = y[2 * i];
            yo[i] = y[2 * i + 1];
        }
        jam_inv<H>(ye, u);
        jam_inv<H>(yo, v);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            x[i] = u[i] + v[i];
            x[N - 1 - i] = u[i] - v[i];
        }
    }
}

// Zig-zag position of coefficient (k, l) of an N x N block (JPEG scan: on odd
// anti-diagonals the row index increases).
template <int N>
__device__ __forceinline__ int zz_pos(int k, int l) {
    const int d = k + l;
    if (d < N) return d * (d + 1) / 2 + ((d & 1) ? k : l);
    const int e = 2 * N - 1 - d;
    return N * N - e * (e + 1) / 2 + ((d & 1) ? k - (d - N + 1) : N - 1 - k);
}

// Row-norm class of row k: n_k = c d[(k >> SH) & 3], d = (4, 9, 10, 9), with
// c = 4, SH = 1 for N = 16 and c = 8, SH = 2 for N = 32.  Returns 0, 1, 2 for
// d = 4, 9, 10.
template <int N>
__host__ __device__ constexpr int norm_class(int k) {
    const int i = (k >> (N == 16 ? 1 : 2)) & 3;
    return i == 0 ? 0 : i == 2 ? 2 : 1;
}

// ------------------------------------------------------------------ arguments

struct JamPlane {
    int64_t in_off, out_off;
    int32_t pitch_in, pitch_out;
    int32_t H, W;
    int32_t nbx;          // blocks per block-row (the last may be partial)
    int32_t tpr;          // tiles per block-row
    int32_t tile_start;   // first tile of the plane inside a frame
    int32_t block_off;    // first block of the plane inside a frame
    uint32_t tpr_m;       // i / tpr = umulhi(i, tpr_m) >> tpr_s (magic_u31)
    int32_t tpr_s;
};

struct JamArgs {
    const uint8_t *in;
    uint8_t *out;
    int32_t *coef;
    unsigned long long *sse;
    int64_t fs_in, fs_out;
    int32_t n_frames, n_planes;
    int32_t tiles_per_frame, blocks_per_frame;
    uint32_t tpf_m;       // g / tiles_per_frame by multiply-high (magic_u31)
    int32_t tpf_s;
    int32_t r, band;      // prefix length, the last anti-diagonal it reaches (at most N - 1)
    int32_t step;
    double inv_step;
    double step_d;
    double skl[3][3];     // 1 / sqrt(n_k n_l) by (class of k, class of l)
    int32_t mu[3][3];     // sqrt(n_k n_l) where it is an integer, else 0
    float qc1[3][3];      // where n_k n_l = mu^2, d = step mu: 1 / d, else 0
    float qc2[3][3];      //   and (d + 1/2) / (2 d)
    int32_t cexact[3];    // L1 / n_k by class (exact inverse, no quantiser)
    double L;             // L1^2
    double inv_L;
    JamPlane pl[kMaxPlanes];
};

// ------------------------------------------------------------------ helpers

// round-half-to-even(n / L) clipped to [0, 255] for an integer n held exactly
// in a double (|n| < 2^53).
__device__ __forceinline__ int rne_div_exact(double n, double L, double inv_L) {
    const double c = fmin(fmax(n, 0.0), 255.0 * L);
    double q = floor(c * inv_L);
    double rem = c - q * L;                 // exact: integers below 2^53
    if (rem < 0.0) { q -= 1.0; rem += L; }
    if (rem >= L) { q += 1.0; rem -= L; }
    const double twice = rem + rem;
    const int qi = int(q);
    return qi + ((twice > L || (twice == L && (qi & 1))) ? 1 : 0);
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) { return wave_sum_u32(v); }

struct JTile {
    int f, p, by, tx;     // frame, plane, block-row, tile inside the block-row
};

// n / d for 0 <= n < 2^31 from the magic pair of a wave-uniform d
__device__ __forceinline__ int udiv_magic(int n, uint32_t m, int s) {
    return s < 0 ? n : int(__umulhi(uint32_t(n), m) >> s);
}

// g is wave-uniform, and so is everything here: multiply-high divisions by
// host-computed magic numbers keep the walk on the scalar unit.
__device__ __forceinline__ JTile jtile_of(const JamArgs &a, int g) {
    JTile t;
    // (the readfirstlanes keep the values scalar where the compiler has moved
    // kernel arguments to vector registers)
    t.f = __builtin_amdgcn_readfirstlane(udiv_magic(g, a.tpf_m, a.tpf_s));
    const int w = __builtin_amdgcn_readfirstlane(g - t.f * a.tiles_per_frame);
    int p = 0;
    while (p + 1 < a.n_planes && w >= a.pl[p + 1].tile_start) ++p;
    t.p = __builtin_amdgcn_readfirstlane(p);
    const JamPlane &P = a.pl[t.p];
    const int i = w - P.tile_start;
    t.by = __builtin_amdgcn_readfirstlane(udiv_magic(i, P.tpr_m, P.tpr_s));
    t.tx = i - t.by * P.tpr;
    return t;
}

// ------------------------------------------------------------------ kernel

// Where one lane's row of one tile lives.
template <int N>
struct JRow {
    int f, p, by, bx, x0, y;
    bool active, full;
};

template <int N>
__device__ __forceinline__ JRow<N> jrow_of(const JamArgs &a, int g, int b, int j) {
    constexpr int WB = 64 / N;
    const JTile t = jtile_of(a, g);
    const JamPlane &Pl = a.pl[t.p];
    JRow<N> r;
    r.f = t.f;
    r.p = t.p;
    r.by = t.by;
    r.bx = t.tx * WB + b;
    r.active = r.bx < Pl.nbx;
    r.x0 = (r.active ? r.bx : Pl.nbx - 1) * N;   // idle lanes read the last block
    r.y = t.by * N + j;
    r.full = r.x0 + N <= Pl.W;
    return r;
}

// The lane's N pixels (rows and columns past the plane repeat its last ones).
template <int N>
__device__ __forceinline__ void load_row(const JamArgs &a, const JRow<N> &r, uint32_t (&pix)[N / 4]) {
    const JamPlane &Pl = a.pl[r.p];
    // a wave-uniform plane base and a 32-bit offset inside the plane (the host
    // bounds H, the pitch and the plane size)
    const uint8_t *src = a.in + int64_t(r.f) * a.fs_in + Pl.in_off +
                         __umul24(uint32_t(min(r.y, Pl.H - 1)), uint32_t(Pl.pitch_in));
    if (r.full) {
#pragma unroll
        for (int v = 0; v < N / 16; ++v) {
            const u32x4 w = __builtin_nontemporal_load((const u32x4 *)(src + r.x0 + 16 * v));
            pix[4 * v] = w.x;
            pix[4 * v + 1] = w.y;
            pix[4 * v + 2] = w.z;
            pix[4 * v + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int v = 0; v < N / 4; ++v) {
            uint32_t w = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) w |= uint32_t(src[min(r.x0 + 4 * v + m, Pl.W - 1)]) << (8 * m);
            pix[v] = w;
        }
    }
}

// Per-lane constants of the lane's column l (row-norm class of l fixed).
struct ColConst {
    double sk[3];     // s_k s_l / step by class of k (quantiser estimate)
    double dq[3];     // step s_k s_l (dequantisation)
    float c1[3], c2[3];   // 1 / d, (d + 1/2) / (2 d) where n_k n_l = mu^2, d = step mu; c1 = 0 elsewhere
    int cex[3];       // L1 / n_k (exact inverse)
    int cexl;         // L1 / n_l
    uint32_t keep;    // bit k: coefficient (k, l) is inside the zig-zag prefix
};

template <int N, int BAND, bool QUANT>
__device__ __forceinline__ void process_tile(const JamArgs &a, const JRow<N> &rw, const uint32_t (&pix)[N / 4],
                                             const ColConst &cc, int32_t *zs, double *us, int lane, int b,
                                             int j, unsigned long long &acc, int &acc_fp) {
    constexpr int NW = N / 4;
    constexpr int P = (BAND + 1) | 1;     // odd LDS row length: conflict-free columns
    const JamPlane &Pl = a.pl[rw.p];

    // ---- row transform; the columns 0..band go to LDS
    {
        int xin[N], z[N];
#pragma unroll
        for (int m = 0; m < N; ++m) xin[m] = int((pix[m >> 2] >> (8 * (m & 3))) & 0xffu);
        jam_fwd<N>(xin, z);
        __syncthreads();                  // the previous tile's readers are done
#pragma unroll
        for (int l = 0; l < N; ++l)
            if (l <= BAND) zs[lane * P + l] = z[l];
    }
    __syncthreads();

    // ---- column transform, zonal prefix, quantiser, column inverse
    {
        const int l = j;
        const int lc = min(l, P - 1);
        int col[N], Y[N];
#pragma unroll
        for (int x = 0; x < N; ++x) col[x] = zs[(b * N + x) * P + lc];
        jam_fwd<N>(col, Y);
        double B[N], U[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            B[k] = 0.0;
            if (k > BAND) continue;       // no column keeps row k
            const int ck = norm_class<N>(k);
            const bool keep = (cc.keep >> k) & 1u;
            int q = Y[k];
            if constexpr (QUANT) {
                // round-half-away(Y s_k s_l / step).  Where n_k n_l = mu^2 the
                // quotient is Y / d, d = step mu, and can be an exact half: there the
                // magnitude floor((2|Y| + d + 1/2) / (2d)) is taken in float32, whose
                // argument lies at least 1/(4d) from an integer while the rounded
                // constants and the fma err by less than (2x + 1) 2^-24 with
                // x < |Y| / d + 1, which is below 1/(4d) as 8|Y| + 12 d < 2^24 (checked
                // on the host); the sign is copied on and the float truncated.
                // Elsewhere the quotient is irrational, never a half, and the nearest
                // integer of its float64 value is right.
                const int mi = __double2loint(fma(double(q), cc.sk[ck], 6755399441055744.0));
                const float yf = float(q);
                const int mr = int(copysignf(fmaf(fabsf(yf), cc.c1[ck], cc.c2[ck]), yf));
                const int m = cc.c1[ck] != 0.f ? mr : mi;
                q = keep ? m : 0;
                B[k] = double(q) * cc.dq[ck];
            } else {
                q = keep ? q : 0;
                B[k] = double(q * cc.cex[ck]) * double(cc.cexl);
            }
            if (a.coef && keep && rw.active) {
                const int64_t gblk = int64_t(rw.f) * a.blocks_per_frame + Pl.block_off +
                                     int64_t(rw.by) * Pl.nbx + rw.bx;
                a.coef[gblk * a.r + zz_pos<N>(k, l)] = q;
            }
        }
        jam_inv<N>(B, U);
        if (j < P) {
#pragma unroll
            for (int x = 0; x < N; ++x) us[(b * N + x) * P + j] = U[x];
        }
    }
    __syncthreads();

    // ---- row inverse, rounding, store, squared error
    double V[N], A[N];
#pragma unroll
    for (int l = 0; l < N; ++l) V[l] = (l <= BAND) ? us[lane * P + l] : 0.0;
    jam_inv<N>(V, A);
    uint32_t o[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) o[v] = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        int px;
        if constexpr (QUANT) px = min(max(__double2loint(A[m] + 6755399441055744.0), 0), 255);
        else px = rne_div_exact(A[m], a.L, a.inv_L);
        o[m >> 2] |= uint32_t(px) << (8 * (m & 3));
    }
    // 32-point: the four lanes that hold image rows j and j + 16 of the tile
    // (lanes j, j + 16 of the left block, j + 32, j + 48 of the right block,
    // j < 16) trade 16-byte quarters, so that each store instruction writes 16
    // whole 64-byte rows: after v_permlane16_swap (which exchanges the odd
    // 16-lane rows of its first operand with the even rows of its second) a lane
    // holds in sx the quarter 2 b + h of row j and in sy that of row j + 16
    // (h = lane / 16 % 2).  Not in the wide-band kernels, which have no
    // registers to spare.
    uint32_t sx[4] = {0u, 0u, 0u, 0u}, sy[4] = {0u, 0u, 0u, 0u};
    bool paired = false;                  // both blocks of the tile inside the plane (wave-uniform)
    if constexpr (N == 32 && BAND < N - 1) {
        paired = (rw.bx | 1) * N + N <= Pl.W;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const auto sw = __builtin_amdgcn_permlane16_swap(o[k], o[4 + k], false, false);
            sx[k] = sw[0];
            sy[k] = sw[1];
        }
    }
    unsigned e = 0;
    if (rw.active && rw.y < Pl.H) {
        // squared error from byte dot products, bytes past the plane masked off:
        // sum (q - a)^2 = sum q^2 + sum a^2 - 2 sum q a
        const int ncol = min(N, Pl.W - rw.x0);
        unsigned sq = 0, cross = 0;
        if (rw.full) {                     // the whole row lies inside the plane
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                sq = __builtin_amdgcn_udot4(o[v], o[v], sq, false);
                sq = __builtin_amdgcn_udot4(pix[v], pix[v], sq, false);
                cross = __builtin_amdgcn_udot4(o[v], pix[v], cross, false);
            }
        } else {
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                const int nb = min(max(ncol - 4 * v, 0), 4);
                const uint32_t msk = nb >= 4 ? 0xffffffffu : ((1u << (8 * nb)) - 1u);
                const uint32_t ov = o[v] & msk, pv = pix[v] & msk;
                sq = __builtin_amdgcn_udot4(ov, ov, sq, false);
                sq = __builtin_amdgcn_udot4(pv, pv, sq, false);
                cross = __builtin_amdgcn_udot4(ov, pv, cross, false);
            }
        }
        e = sq - 2u * cross;
        if (a.out && !paired) {
            uint8_t *dst = a.out + int64_t(rw.f) * a.fs_out + Pl.out_off +
                           (__umul24(uint32_t(rw.y), uint32_t(Pl.pitch_out)) + uint32_t(rw.x0));
            if (rw.full) {
#pragma unroll
                for (int v = 0; v < NW / 4; ++v) {
                    u32x4 w;
                    w.x = o[4 * v];
                    w.y = o[4 * v + 1];
                    w.z = o[4 * v + 2];
                    w.w = o[4 * v + 3];
                    __builtin_nontemporal_store(w, (u32x4 *)(dst + 16 * v));
                }
            } else {
#pragma unroll
                for (int m = 0; m < N; ++m)
                    if (m < ncol) dst[m] = uint8_t(o[m >> 2] >> (8 * (m & 3)));
            }
        }
    }
    if (paired && a.out) {
        const int h = (lane >> 4) & 1;
        const int y1 = rw.y - 16 * h;     // row j of the tile (j = lane % 16)
        uint8_t *p1 = a.out + int64_t(rw.f) * a.fs_out + Pl.out_off +
                      (__umul24(uint32_t(y1), uint32_t(Pl.pitch_out)) + uint32_t(rw.x0 + 16 * h));
        if (y1 < Pl.H) __builtin_nontemporal_store(u32x4{sx[0], sx[1], sx[2], sx[3]}, (u32x4 *)p1);
        if (y1 + 16 < Pl.H)
            __builtin_nontemporal_store(u32x4{sy[0], sy[1], sy[2], sy[3]},
                                        (u32x4 *)(p1 + 16 * uint32_t(Pl.pitch_out)));
    }
    // squared errors: one atomic per (frame, plane) run of the wave
    const int fp = rw.f * a.n_planes + rw.p;
    if (fp != acc_fp) {
        if (acc_fp >= 0 && acc && lane == 0) atomicAdd(a.sse + acc_fp, acc);
        acc = 0;
        acc_fp = fp;
    }
    acc += wave_sum(e);
}

// The 16-point narrow-band kernel is held to 128 VGPRs (4 waves per SIMD; a few
// bytes spill), which pays; the others would spill heavily.
template <int N, int BAND, bool QUANT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(N == 16 && BAND <= 8 ? 4 : 1, 8))) void k_jam(const JamArgs a) {
    constexpr int NW = N / 4;
    constexpr int P = (BAND + 1) | 1;
    // two LDS areas, so that the column pass can store its inverse while other
    // lanes may still be reading their columns: rows of the forward pass (int32)
    // and columns of the inverse (double), both 64 x P
    extern __shared__ double lds_raw[];
    const int lane = threadIdx.x;
    const int b = lane / N, j = lane - b * N;     // block in tile, row (then column)
    const int total = a.n_frames * a.tiles_per_frame;
    int32_t *zs = reinterpret_cast<int32_t *>(lds_raw);
    double *us = lds_raw + 32 * P;

    // constants of the lane's column l = j
    ColConst cc;
    {
        const int cl = norm_class<N>(j);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double skl = cl == 0 ? a.skl[c][0] : cl == 1 ? a.skl[c][1] : a.skl[c][2];
            cc.sk[c] = skl * a.inv_step;
            cc.dq[c] = skl * a.step_d;
            cc.c1[c] = cl == 0 ? a.qc1[c][0] : cl == 1 ? a.qc1[c][1] : a.qc1[c][2];
            cc.c2[c] = cl == 0 ? a.qc2[c][0] : cl == 1 ? a.qc2[c][1] : a.qc2[c][2];
            cc.cex[c] = a.cexact[c];
        }
        cc.cexl = cl == 0 ? a.cexact[0] : cl == 1 ? a.cexact[1] : a.cexact[2];
        cc.keep = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) cc.keep |= (zz_pos<N>(k, j) < a.r) ? (1u << k) : 0u;
    }

    unsigned long long acc = 0;
    int acc_fp = -1;
    int g = blockIdx.x;
    if (g >= total) return;
    // the next tile's row loads are issued before the current tile is processed,
    // on every pass (the last pass re-reads its own tile), so no branch joins
    // paths with loads in flight
    uint32_t pa[NW], pb[NW];
    JRow<N> ra = jrow_of<N>(a, g, b, j), rb = ra;
    load_row<N>(a, ra, pa);
    while (true) {
        int nx = g + int(gridDim.x);
        bool more = nx < total;
        rb = jrow_of<N>(a, more ? nx : g, b, j);
        load_row<N>(a, rb, pb);
        process_tile<N, BAND, QUANT>(a, ra, pa, cc, zs, us, lane, b, j, acc, acc_fp);
        if (!more) break;
        g = nx;
        nx = g + int(gridDim.x);
        more = nx < total;
        ra = jrow_of<N>(a, more ? nx : g, b, j);
        load_row<N>(a, ra, pa);
        process_tile<N, BAND, QUANT>(a, rb, pb, cc, zs, us, lane, b, j, acc, acc_fp);
        if (!more) break;
        g = nx;
    }
    if (acc_fp >= 0 && acc && lane == 0) atomicAdd(a.sse + acc_fp, acc);
}

__global__ void k_jam_zero(unsigned long long *p, int n) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0ull;
}

template <int N, int BAND, bool QUANT>
adct_status launch(const JamArgs &a, hipStream_t s) {
    auto kern = k_jam<N, BAND, QUANT>;
    constexpr int P = (BAND + 1) | 1;
    const size_t lds = size_t(64) * P * (sizeof(int32_t) + sizeof(double));
    int dev = 0, cus = 0, per_cu = 0;
    ADCT_HIP(hipGetDevice(&dev));
    ADCT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds));
    if (per_cu < 1) per_cu = 1;
    const int64_t tiles = int64_t(a.n_frames) * a.tiles_per_frame;
    const int grid = int(std::min<int64_t>(tiles, int64_t(per_cu) * cus));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, s, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

// ------------------------------------------------------------------ host matrices

// T_(N) grown from the 8-point T1 by the construction of Sec. 6.2, in the sign
// convention of the printed matrices: row 2i = [t_i, rev(t_i)], row 2i + 1 =
// [t_i, -rev(t_i)].
void jam_matrix_host(int N, int8_t *T) {
    int8_t cur[32 * 32], nxt[32 * 32];
    int h = 8;
    for (int k = 0; k < 8; ++k)
        for (int m = 0; m < 8; ++m) cur[k * 8 + m] = kT1.m[k][m];
    while (h < N) {
        const int n = 2 * h;
        for (int i = 0; i < h; ++i)
            for (int m = 0; m < h; ++m) {
                const int8_t v = cur[i * h + m], w = cur[i * h + (h - 1 - m)];
                nxt[(2 * i) * n + m] = v;
                nxt[(2 * i) * n + h + m] = w;
                nxt[(2 * i + 1) * n + m] = v;
                nxt[(2 * i + 1) * n + h + m] = int8_t(-w);
            }
        memcpy(cur, nxt, size_t(n) * n);
        h = n;
    }
    memcpy(T, cur, size_t(N) * N);
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" adct_status adct_jam_matrix(adct_transform_id base, int N, int8_t *T, int32_t *n) {
    if (!T || !n) return fail(ADCT_EINVAL, "T and n are required");
    if (base != ADCT_T1) return fail(ADCT_ENOTSUP, "the JAM matrices are built from T1 only");
    if (N != 16 && N != 32) return fail(ADCT_ERANGE, "N must be 16 or 32");
    jam_matrix_host(N, T);
    for (int k = 0; k < N; ++k) {
        int32_t s = 0;
        for (int m = 0; m < N; ++m) s += int32_t(T[k * N + m]) * T[k * N + m];
        n[k] = s;
    }
    return ADCT_OK;
}

extern "C" adct_status adct_jam_evaluate_stream(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                                const adct_plane *planes, int n_planes,
                                                adct_transform_id base, int N, int r, int quant_step,
                                                int32_t *coef, uint8_t *recon, int64_t frame_stride_out,
                                                uint64_t *sse, adct_stream_t stream) {
    if (!frames || !planes || !sse) return fail(ADCT_EINVAL, "frames, planes and sse are required");
    if (base != ADCT_T1) return fail(ADCT_ENOTSUP, "the JAM matrices are built from T1 only");
    if (N != 16 && N != 32) return fail(ADCT_ERANGE, "N must be 16 or 32");
    if (r < 1 || r > N * N) return fail(ADCT_ERANGE, "r must be in [1, N*N]");
    if (quant_step < 0 || quant_step > 4096) return fail(ADCT_ERANGE, "quant_step must be in [0, 4096]");
    if (quant_step % N)
        return fail(ADCT_ENOTSUP, "quant_step must be a multiple of N (a reconstruction could sit on an exact half)");
    if (n_frames < 1) return fail(ADCT_ERANGE, "n_frames must be >= 1");
    if (n_planes < 1 || n_planes > kMaxPlanes) return fail(ADCT_ERANGE, "n_planes must be in [1, 4]");
    if (n_frames > 1 && frame_stride <= 0) return fail(ADCT_EDIM, "frame_stride must be positive for several frames");
    if (recon && n_frames > 1 && frame_stride_out <= 0)
        return fail(ADCT_EDIM, "frame_stride_out must be positive for several frames");
    if ((reinterpret_cast<uintptr_t>(sse) & 7) || (reinterpret_cast<uintptr_t>(coef) & 3))
        return fail(ADCT_EDIM, "sse must be 8-byte and coef 4-byte aligned");
    JamArgs a;
    memset(&a, 0, sizeof(a));
    a.in = frames;
    a.out = recon;
    a.coef = coef;
    a.sse = reinterpret_cast<unsigned long long *>(sse);
    a.fs_in = frame_stride;
    a.fs_out = frame_stride_out;
    a.n_frames = n_frames;
    a.n_planes = n_planes;
    const int WB = 64 / N;
    int64_t tiles = 0, blocks = 0;
    for (int p = 0; p < n_planes; ++p) {
        const adct_plane &q = planes[p];
        if (q.H < 1 || q.W < 1 || q.pitch < q.W || q.offset < 0)
            return fail(ADCT_EDIM, "each plane needs H, W >= 1, pitch >= W and offset >= 0");
        if (q.H >= (1 << 24) || q.pitch >= (1 << 24) || int64_t(q.H) * q.pitch >= (int64_t(1) << 31))
            return fail(ADCT_ERANGE, "planes are limited to H, pitch < 2^24 and H * pitch < 2^31");
        JamPlane &d = a.pl[p];
        d.in_off = q.offset;
        d.out_off = q.offset;
        d.pitch_in = q.pitch;
        d.pitch_out = q.pitch;
        d.H = q.H;
        d.W = q.W;
        d.nbx = (q.W + N - 1) / N;
        d.tpr = (d.nbx + WB - 1) / WB;
        d.tile_start = int32_t(tiles);
        d.block_off = int32_t(blocks);
        magic_u31(uint32_t(d.tpr), &d.tpr_m, &d.tpr_s);
        const int64_t nby = (q.H + N - 1) / N;
        tiles += nby * d.tpr;
        blocks += nby * d.nbx;
        if (tiles > (int64_t(1) << 30) || blocks > (int64_t(1) << 30))
            return fail(ADCT_ERANGE, "plane too large");
    }
    if (tiles * n_frames > (int64_t(1) << 31) - 1 || blocks * n_frames * r > (int64_t(1) << 40))
        return fail(ADCT_ERANGE, "too many blocks in one call");
    a.tiles_per_frame = int32_t(tiles);
    a.blocks_per_frame = int32_t(blocks);
    magic_u31(uint32_t(tiles), &a.tpf_m, &a.tpf_s);
    a.r = r;
    // last anti-diagonal reached by the prefix of length r
    int band = 0, cnt = 0;
    for (int d = 0; d < 2 * N - 1; ++d) {
        cnt += d < N ? d + 1 : 2 * N - 1 - d;
        if (cnt >= r) {
            band = d;
            break;
        }
    }
    a.band = std::min(band, N - 1);
    a.step = quant_step;
    a.step_d = double(quant_step);
    a.inv_step = quant_step ? 1.0 / double(quant_step) : 0.0;
    const int c = N == 16 ? 4 : 8;
    const int dv[3] = {4, 9, 10};
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            const int64_t v = int64_t(c) * dv[i] * c * dv[k];
            int32_t m = 0;
            for (int32_t s = 1; int64_t(s) * s <= v; ++s)
                if (int64_t(s) * s == v) m = s;
            a.mu[i][k] = m;
            a.skl[i][k] = 1.0 / sqrt(double(v));
            const double d = double(m) * quant_step;
            a.qc1[i][k] = m && quant_step ? float(1.0 / d) : 0.f;
            a.qc2[i][k] = m && quant_step ? float((d + 0.5) / (2.0 * d)) : 0.f;
        }
    // the float32 quantiser of the classes with exact halves needs 8 |Y| + 12 d < 2^24
    // (|Y| <= 255 (max row sum of |T|)^2, d = step mu)
    if (quant_step) {
        int8_t T[32 * 32];
        jam_matrix_host(N, T);
        int64_t rs = 0;
        for (int k = 0; k < N; ++k) {
            int64_t s = 0;
            for (int m = 0; m < N; ++m) s += std::abs(int(T[k * N + m]));
            rs = std::max(rs, s);
        }
        int64_t mu_max = 0;
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) mu_max = std::max<int64_t>(mu_max, a.mu[i][k]);
        if (8 * 255 * rs * rs + 12 * mu_max * quant_step >= (int64_t(1) << 24))
            return fail(ADCT_ERANGE, "quant_step too large for the exact quantiser");
    }
    const int64_t L1 = int64_t(c) * 4 * 9 * 10 / 2;   // lcm(4c, 9c, 10c) = 180 c
    for (int i = 0; i < 3; ++i) a.cexact[i] = int32_t(L1 / (int64_t(c) * dv[i]));
    a.L = double(L1) * double(L1);
    a.inv_L = 1.0 / a.L;
    for (int p = 0; p < n_planes; ++p) {
        a.pl[p].pitch_out = recon ? planes[p].pitch : 0;
    }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int nz = n_frames * n_planes;
    hipLaunchKernelGGL(k_jam_zero, dim3((nz + 255) / 256), dim3(256), 0, hs, a.sse, nz);
    ADCT_HIP(hipGetLastError());
    // kernels for the band of the prefix (rows and columns past it are known
    // zeros at compile time): N = 16 up to r = 45 and N = 32 up to r = 171, or any r
    if (N == 16) {
        if (a.band <= 8) return quant_step ? launch<16, 8, true>(a, hs) : launch<16, 8, false>(a, hs);
        return quant_step ? launch<16, 15, true>(a, hs) : launch<16, 15, false>(a, hs);
    }
    if (a.band <= 17) return quant_step ? launch<32, 17, true>(a, hs) : launch<32, 17, false>(a, hs);
    return quant_step ? launch<32, 31, true>(a, hs) : launch<32, 31, false>(a, hs);
}
