// Batched evaluation: many images of uneven sizes x several transforms x every
// retention level r in one persistent launch per arithmetic (the rate-distortion
// sweep of Sec. 6.1.1, where the paper averages MSE / PSNR over images for each
// r).
//
// A work item is one tile of 64 blocks of one image and a group of transforms;
// one wave owns an item, one lane owns one block.  Per transform the lane
// computes the forward transform once, stages its coefficients in LDS (zig-zag
// order, lane-interleaved so every read is conflict-free), then walks the
// zig-zag scan: step j adds coefficient j's outer product to the block's
// reconstruction numerator, rounds, clips and scores it, giving the squared
// error for r = j + 1.  Each step's per-lane errors are summed across the wave
// and added to the [image][transform][r] table.
//
// Integer transforms accumulate exact integer numerators over L = lcm(n)^2
// (bit-exact against the oracle).  Their coefficients are staged as int16 (8 KB
// per wave), so many waves share a compute unit and hide each other's latency.
// The exact DCT accumulates in float64 and stages float64 coefficients (32 KB per
// wave); it runs as a second kernel so that its LDS footprint does not cap the
// occupancy of the integer sweep.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr int kMaxBatchImages = 64;
constexpr int kMaxBatchTransforms = 8;

struct BatchImg {
    int64_t offset;
    int32_t pitch;
    int32_t nbx;
    int32_t nblocks;
    int32_t tile_start;    // first tile of this image in the global tile order
};

struct BatchArgs {
    const uint8_t *base;
    unsigned long long *sse;          // [image][transform][r - r_lo]
    int32_t n_images;
    int32_t n_transforms;
    int32_t r_lo, r_hi;
    int32_t split;                    // integer-transform groups per tile
    int32_t total_tiles;
    int32_t tids[kMaxBatchTransforms];
    int32_t n_int, n_dct;             // integer / DCT entries of the list
    int32_t int_pos[kMaxBatchTransforms];   // their positions in the list
    int32_t dct_pos[kMaxBatchTransforms];
    BatchImg img[kMaxBatchImages];
};

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// cos(m pi / 16) by its Taylor series (exact to the last bit for |x| <= pi)
constexpr double ccos(double x) {
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 40; ++i) {
        term *= -x * x / ((2 * i - 1) * (2 * i));
        sum += term;
    }
    return sum;
}
struct DctTab {
    double c[64];     // orthonormal DCT-II, c[8k + x] = a_k cos((2x+1) k pi / 16)
};
constexpr DctTab make_dct() {
    DctTab t{};
    constexpr double pi = 3.14159265358979323846;
    for (int k = 0; k < 8; ++k)
        for (int x = 0; x < 8; ++x) {
            int m = ((2 * x + 1) * k) % 32;               // angle m pi / 16 in [0, 2 pi)
            double sgn = 1.0;
            if (m > 16) m = 32 - m;                       // cos(2 pi - a) = cos a
            if (m > 8) {                                  // cos(pi - a) = -cos a
                m = 16 - m;
                sgn = -1.0;
            }
            const double alpha = k == 0 ? 0.35355339059327376220 : 0.5;
            t.c[8 * k + x] = sgn * alpha * ccos(m * pi / 16.0);
        }
    return t;
}
__device__ constexpr DctTab kDct = make_dct();

// device-resident copies of the tables indexed by run-time (wave-uniform) values
struct ZZTab {
    int8_t k[64], l[64];     // row / column of the z-th zig-zag coefficient
};
constexpr ZZTab make_zz() {
    ZZTab t{};
    for (int z = 0; z < 64; ++z) {
        t.k[z] = int8_t(kZZ[z] >> 3);
        t.l[z] = int8_t(kZZ[z] & 7);
    }
    return t;
}
__device__ constexpr ZZTab kZZDev = make_zz();
__device__ constexpr Mat8 kMatDev[7] = {kT1, kT1, kT2, kLOx2, kT6, kRDCT, kT4};

// packed 8-bit reconstruction row -> squared-error terms (see emit_row)
__device__ __forceinline__ void score_row(const int (&q)[8], uint32_t w0, uint32_t w1, uint32_t &sq,
                                          uint32_t &cross) {
    const uint32_t r01 = uint32_t(q[0]) | (uint32_t(q[1]) << 16);
    const uint32_t r23 = uint32_t(q[2]) | (uint32_t(q[3]) << 16);
    const uint32_t r45 = uint32_t(q[4]) | (uint32_t(q[5]) << 16);
    const uint32_t r67 = uint32_t(q[6]) | (uint32_t(q[7]) << 16);
    const uint32_t lo = __builtin_amdgcn_perm(r23, r01, 0x06040200u);
    const uint32_t hi = __builtin_amdgcn_perm(r67, r45, 0x06040200u);
    sq = __builtin_amdgcn_udot4(lo, lo, sq, false);
    sq = __builtin_amdgcn_udot4(hi, hi, sq, false);
    cross = __builtin_amdgcn_udot4(lo, w0, cross, false);
    cross = __builtin_amdgcn_udot4(hi, w1, cross, false);
}

// sum of squared pixels of a block (constant across r)
__device__ __forceinline__ uint32_t pix_energy(const uint32_t (&pix)[8][2]) {
    uint32_t e = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        e = __builtin_amdgcn_udot4(pix[x][0], pix[x][0], e, false);
        e = __builtin_amdgcn_udot4(pix[x][1], pix[x][1], e, false);
    }
    return e;
}

__device__ __forceinline__ unsigned wave_add(unsigned v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int pix_at(const uint32_t (&pix)[8][2], int x, int y) {
    return int((pix[x][y >> 2] >> (8 * (y & 3))) & 0xffu);
}

// 8-point forward y = T x, all 8 outputs (even/odd butterfly on compile-time T)
template <int ID>
__device__ __forceinline__ void fwd_full(const int (&x)[8], int (&y)[8]) {
    int s[4], d[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        s[m] = x[m] + x[7 - m];
        d[m] = x[m] - x[7 - m];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int acc = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) acc += Tf<ID>::t(k, m) * ((k & 1) ? d[m] : s[m]);
        y[k] = acc;
    }
}

// ---------------------------------------------------------------- integer sweep
//
// Step j of the scan adds the coefficient at zig-zag position j, (k, l):
//     A[x][y] += V(k,l) T[k][x] T[l][y],   V = Y c_k c_l,  Y = T A T^T.
// With g_k the gcd of row k's entries, Y' = Y / (g_k g_l) fits int16 for 8-bit
// input, and the step becomes two 24-bit products per entry:
//     u[x] = Y' T[k][x],   A[x][y] += u[x] w_y,   w_y = g_k g_l c_k c_l T[l][y].
// The sixteen wave-uniform factors of a step sit in one table row (one scalar
// load), so the step has no branches.

struct StepEnt {
    int16_t w[8];     // g_k g_l c_k c_l T[l][y]
    int16_t tk[8];    // T[k][x]
};
struct StepTab {
    StepEnt s[64];
};

template <int ID>
constexpr int32_t row_gcd(int k) {
    int32_t g = 0;
    for (int m = 0; m < 8; ++m) {
        int32_t v = Tf<ID>::t(k, m) < 0 ? -Tf<ID>::t(k, m) : Tf<ID>::t(k, m);
        int32_t a = g;
        while (v) {
            const int32_t r = a % v;
            a = v;
            v = r;
        }
        g = a;
    }
    return g;
}

constexpr int32_t log2_exact(int32_t v) {
    int32_t s = 0;
    while ((1 << s) < v) ++s;
    return (1 << s) == v ? s : -1;
}

template <int ID>
constexpr StepTab make_steps() {
    StepTab t{};
    for (int j = 0; j < 64; ++j) {
        const int k = kZZ[j] >> 3, l = kZZ[j] & 7;
        const int32_t g = row_gcd<ID>(k) * row_gcd<ID>(l);
        for (int x = 0; x < 8; ++x) {
            t.s[j].tk[x] = int16_t(Tf<ID>::t(k, x));
            t.s[j].w[x] = int16_t(g * Tf<ID>::c(k) * Tf<ID>::c(l) * Tf<ID>::t(l, x));
        }
    }
    return t;
}

// log2 of each row's gcd (a power of two for every built-in transform)
template <int ID>
struct RowShift {
    struct Tab {
        int32_t sh[8];
    };
    static constexpr Tab make() {
        Tab t{};
        for (int k = 0; k < 8; ++k) t.sh[k] = log2_exact(row_gcd<ID>(k));
        return t;
    }
    static constexpr Tab kT = make();
};

// Range facts the integer sweep relies on, checked at compile time:
//  * |Y'| <= 32767: the largest |Y(k,l)| over 8-bit blocks is 255 times the
//    larger of the positive and negative parts of the outer product of rows k, l;
//  * u fits signed 24 bits, w signed 16 bits, and |u w| < 2^31;
//  * 2L fits signed 24 bits (the tie test multiplies it by the quotient).
// The numerator itself stays below 2040 L in magnitude: every prefix of the scan
// is an orthogonal projection of the block, whose norm is at most 255 * 8.
template <int ID>
constexpr bool int_sweep_ranges_ok() {
    int64_t umax = 0, wmax = 0;
    for (int k = 0; k < 8; ++k)
        for (int l = 0; l < 8; ++l) {
            int64_t pos = 0, neg = 0;
            for (int x = 0; x < 8; ++x)
                for (int y = 0; y < 8; ++y) {
                    const int64_t p = int64_t(Tf<ID>::t(k, x)) * Tf<ID>::t(l, y);
                    if (p > 0) pos += p; else neg -= p;
                }
            const int64_t g = int64_t(row_gcd<ID>(k)) * row_gcd<ID>(l);
            if (log2_exact(int32_t(g)) < 0) return false;
            const int64_t ymax = 255 * (pos > neg ? pos : neg) / g;
            if (ymax > 32767) return false;
            for (int x = 0; x < 8; ++x) {
                const int64_t tk = Tf<ID>::t(k, x) < 0 ? -Tf<ID>::t(k, x) : Tf<ID>::t(k, x);
                const int64_t tl = Tf<ID>::t(l, x) < 0 ? -Tf<ID>::t(l, x) : Tf<ID>::t(l, x);
                umax = umax > ymax * tk ? umax : ymax * tk;
                const int64_t w = g * Tf<ID>::c(k) * Tf<ID>::c(l) * tl;
                wmax = wmax > w ? wmax : w;
            }
        }
    const int64_t L = Tf<ID>::L();
    return umax < (1 << 23) && wmax < (1 << 15) && umax * wmax < (int64_t(1) << 31) &&
           2 * L < (1 << 23) && int64_t(2040) * L * 2 + L < (int64_t(1) << 31);
}

__device__ constexpr StepTab kStepDev[7] = {make_steps<ADCT_T1>(), make_steps<ADCT_T1>(),
                                            make_steps<ADCT_T2>(), make_steps<ADCT_LO>(),
                                            make_steps<ADCT_T6>(), make_steps<ADCT_RDCT>(),
                                            make_steps<ADCT_T4>()};
static_assert(int_sweep_ranges_ok<ADCT_T1>() && int_sweep_ranges_ok<ADCT_T2>() &&
                  int_sweep_ranges_ok<ADCT_LO>() && int_sweep_ranges_ok<ADCT_T6>() &&
                  int_sweep_ranges_ok<ADCT_RDCT>() && int_sweep_ranges_ok<ADCT_T4>(),
              "integer sweep ranges");

// Exact round-half-to-even(n / L) clipped to [0, 255] without a 32-bit
// multiply.  With c = clip(n) and u = 2c + L, the half-up quotient is
// q = floor(u / 2L), found in float:
//  * small L: u / 2L = c / L + 1/2 and fma(c, 1/L, 1/2 + 1/(4L)) lies in
//    [q, q + 1): the fractions of u / 2L are multiples of 1/(2L), and the
//    rounding error (below 256 * 2^-23 + 2^-24) is under the 1/(4L) offset;
//  * large L: write 2L = 2^a b with b odd; q = floor(v / b) for
//    v = u >> a = (c + L/2) >> (a - 1), and fma(v, 1/b, 1/(2b)) lies in
//    [q, q + 1) by the same argument with spacing 1/b.
// At a tie u = 2L q, i.e. c + L/2 - L q = 0 (L is even); that remainder is an
// integer in [0, L), so minus one it is negative exactly at a tie, where an odd
// q loses its low bit.
template <int ID>
struct IntRound {
    static constexpr int32_t L = Tf<ID>::L();
    static constexpr bool kShift = L >= 4096;
    static constexpr int32_t a() {
        int32_t s = 0;
        while (((2 * L) >> s & 1) == 0) ++s;
        return s;
    }
    static constexpr int32_t kA = kShift ? a() : 0;
    static constexpr int32_t kB = (2 * L) >> kA;           // odd part of 2L (large L)
    static_assert(!kShift || (kA >= 1 && kB <= 8192), "divisor too large for the float quotient");
    static_assert(kShift || L <= 8192, "small-L path needs 1/(4L) above the rounding error");
    static_assert(int64_t(256) * L < (int64_t(1) << (24 + kA)), "quotient input must be exact in float");
    static_assert(L % 2 == 0, "the tie test halves u");
};

// wave-uniform constants of the rounding, held in scalar registers (a VOP3
// instruction takes no 32-bit literal on this target)
struct IntRoundRegs {
    int32_t hLm1, mL;     // L/2 - 1, -L
};

template <int ID>
__device__ __forceinline__ IntRoundRegs int_round_regs() {
    IntRoundRegs r;
    asm("s_mov_b32 %0, %1" : "=s"(r.hLm1) : "i"(IntRound<ID>::L / 2 - 1));
    asm("s_mov_b32 %0, %1" : "=s"(r.mL) : "i"(-IntRound<ID>::L));
    return r;
}

template <int ID>
__device__ __forceinline__ int rne_clip_int(int n, const IntRoundRegs &c) {
    using R = IntRound<ID>;
    const int nc = min(max(n, 0), 255 * R::L);
    float f;
    if constexpr (R::kShift) {
        constexpr float kInv = 1.0f / float(R::kB);
        constexpr float kOff = 0.5f / float(R::kB);
        f = __builtin_fmaf(float(uint32_t(nc + R::L / 2) >> (R::kA - 1)), kInv, kOff);
    } else {
        constexpr float kInv = 1.0f / float(R::L);
        constexpr float kOff = 0.5f + 0.25f / float(R::L);
        f = __builtin_fmaf(float(nc), kInv, kOff);
    }
    const uint32_t q = uint32_t(f);
    const uint32_t tie = uint32_t(nc + c.hLm1 + __mul24(int(q), c.mL)) >> 31;
    return int(q & ~tie);
}

// Per-wave coefficient staging for the integer sweep: [z][lane] int16.
__shared__ int16_t g_stage16[64 * 64];

// column pass of the forward for column Lc: Y[:, Lc] = T Z[:, Lc]; stores
// Y' = Y / (g_k g_Lc) at the coefficient's zig-zag slot
template <int ID, int Lc>
__device__ __forceinline__ void fwd_col16(const int (&Z)[8][8], int16_t *lds, int lane) {
    int in[8], out[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) in[x] = Z[x][Lc];
    fwd_full<ID>(in, out);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        lds[zz_pos(k, Lc) * 64 + lane] = int16_t(out[k] >> (RowShift<ID>::kT.sh[k] + RowShift<ID>::kT.sh[Lc]));
}

template <int ID, size_t... Ls>
__device__ __forceinline__ void fwd_cols16(const int (&Z)[8][8], int16_t *lds, int lane, std::index_sequence<Ls...>) {
    (fwd_col16<ID, int(Ls)>(Z, lds, lane), ...);
}

// One integer transform's sweep over the zig-zag scan for the lane's block;
// `out` points at the transform's r_lo..r_hi row of the table.
// an empty asm that claims to rewrite the block's words: values derived from
// them cannot be hoisted out of the per-transform loop and kept live across
// every sweep
__device__ __forceinline__ void opaque_block(uint32_t (&pix)[8][2]) {
#pragma unroll
    for (int x = 0; x < 8; ++x) asm volatile("" : "+v"(pix[x][0]), "+v"(pix[x][1]));
}

template <int ID>
__device__ __forceinline__ void sweep_int(const uint32_t (&pix_in)[8][2], bool active, unsigned long long *out,
                                          int r_lo, int r_hi, int lane) {
    uint32_t pix[8][2];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        pix[x][0] = pix_in[x][0];
        pix[x][1] = pix_in[x][1];
    }
    opaque_block(pix);
    int16_t *lds = g_stage16;
    {
        int Z[8][8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int in[8], o[8];
#pragma unroll
            for (int y = 0; y < 8; ++y) in[y] = pix_at(pix, x, y);
            fwd_full<ID>(in, o);
#pragma unroll
            for (int l = 0; l < 8; ++l) Z[x][l] = o[l];
        }
        fwd_cols16<ID>(Z, lds, lane, std::make_index_sequence<8>{});
    }
    __builtin_amdgcn_wave_barrier();
    int A[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) A[x][y] = 0;
    const uint32_t e_pix = pix_energy(pix);
    const StepEnt *S = kStepDev[ID].s;
    const IntRoundRegs rc = int_round_regs<ID>();
    int v = lds[lane];
    for (int j = 0; j < r_hi; ++j) {
        const int vn = lds[((j + 1) & 63) * 64 + lane];     // next step's coefficient
        const StepEnt &E = S[j];                             // wave-uniform: scalar loads
        int u[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) u[x] = v * int(E.tk[x]);
        // operands of known narrow range select the 24-bit multiply(-add)
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y) A[x][y] = __mul24(u[x], int(E.w[y])) + A[x][y];
        uint32_t sq = e_pix, cross = 0;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int q[8];
#pragma unroll
            for (int y = 0; y < 8; ++y) q[y] = rne_clip_int<ID>(A[x][y], rc);
            score_row(q, pix[x][0], pix[x][1], sq, cross);
        }
        unsigned err = sq - 2u * cross;
        if (j + 1 >= r_lo) {
            err = wave_add(active ? err : 0u);
            if (lane == 0 && err) atomicAdd(out + (j + 1 - r_lo), (unsigned long long)err);
        }
        v = vn;
    }
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- float64 DCT sweep
//
// Step j (zig-zag (k, l)) adds B(k,l) C[k][x] C[l][y] to pixel (x, y).  The
// lane keeps 32 float64 accumulators (four pixel rows) per pass, so the block
// takes two passes over the scan; the coefficients are staged in LDS 32 at a
// time (16 KB per wave), each window computed by a column-wise forward that
// keeps one column of the row pass live.  The forward is repeated per pass and
// window (its arithmetic, and so every coefficient, is the same each time).

struct DctStep {
    double ck[8];     // C[k][x]
    double cl[8];     // C[l][y]
};
struct DctStepTab {
    DctStep s[64];
};
constexpr DctStepTab make_dct_steps() {
    DctStepTab t{};
    const DctTab c = make_dct();
    for (int j = 0; j < 64; ++j) {
        const int k = kZZ[j] >> 3, l = kZZ[j] & 7;
        for (int x = 0; x < 8; ++x) {
            t.s[j].ck[x] = c.c[8 * k + x];
            t.s[j].cl[x] = c.c[8 * l + x];
        }
    }
    return t;
}
__device__ constexpr DctStepTab kDctStep = make_dct_steps();

constexpr int kDctWin = 32;                    // coefficients per staged window
__shared__ double g_stage64[kDctWin * 64];     // [z - window start][lane]

// One column Lc of the forward, restricted to window W: the row pass
// Z[x] = sum_y A[x][y] C[Lc][y] (even/odd butterfly, exact integer sums first),
// then B(k, Lc) = sum_x C[k][x] Z[x] for the k whose zig-zag slot is in W.
template <int W, int Lc>
__device__ __forceinline__ void dct_fwd_col(const uint32_t (&pix_in)[8][2], double *lds, int lane) {
    constexpr int lo = W * kDctWin, hi = lo + kDctWin;
    constexpr bool any = (zz_pos(0, Lc) >= lo && zz_pos(0, Lc) < hi) || (zz_pos(1, Lc) >= lo && zz_pos(1, Lc) < hi) ||
                         (zz_pos(2, Lc) >= lo && zz_pos(2, Lc) < hi) || (zz_pos(3, Lc) >= lo && zz_pos(3, Lc) < hi) ||
                         (zz_pos(4, Lc) >= lo && zz_pos(4, Lc) < hi) || (zz_pos(5, Lc) >= lo && zz_pos(5, Lc) < hi) ||
                         (zz_pos(6, Lc) >= lo && zz_pos(6, Lc) < hi) || (zz_pos(7, Lc) >= lo && zz_pos(7, Lc) < hi);
    if constexpr (any) {
        // a fresh opaque copy per column: the butterfly sums shared by columns of
        // equal parity are recomputed rather than kept live across columns
        uint32_t pix[8][2];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            pix[x][0] = pix_in[x][0];
            pix[x][1] = pix_in[x][1];
        }
        opaque_block(pix);
        double Z[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int sd = (Lc & 1) ? pix_at(pix, x, m) - pix_at(pix, x, 7 - m)
                                        : pix_at(pix, x, m) + pix_at(pix, x, 7 - m);
                acc = fma(double(sd), kDct.c[8 * Lc + m], acc);
            }
            Z[x] = acc;
        }
        double se[4], de[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            se[m] = Z[m] + Z[7 - m];
            de[m] = Z[m] - Z[7 - m];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int z = zz_pos(k, Lc);
            if (z >= lo && z < hi) {
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < 4; ++m) acc = fma(kDct.c[8 * k + m], (k & 1) ? de[m] : se[m], acc);
                lds[(z - lo) * 64 + lane] = acc;
            }
        }
    }
}

template <int W, size_t... Ls>
__device__ __forceinline__ void dct_fwd_window(const uint32_t (&pix)[8][2], double *lds, int lane,
                                               std::index_sequence<Ls...>) {
    (dct_fwd_col<W, int(Ls)>(pix, lds, lane), ...);
}

// Exact DCT: float64 incremental reconstruction over the zig-zag scan.
__device__ __forceinline__ void sweep_dct(const uint32_t (&pix_in)[8][2], bool active, unsigned long long *out,
                                          int r_lo, int r_hi, int lane) {
    uint32_t pix[8][2];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        pix[x][0] = pix_in[x][0];
        pix[x][1] = pix_in[x][1];
    }
    opaque_block(pix);
    double *lds = g_stage64;
    const DctStep *S = kDctStep.s;
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        uint32_t rows[4][2];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            rows[x][0] = h ? pix[4 + x][0] : pix[x][0];
            rows[x][1] = h ? pix[4 + x][1] : pix[x][1];
        }
        uint32_t e_half = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            e_half = __builtin_amdgcn_udot4(rows[x][0], rows[x][0], e_half, false);
            e_half = __builtin_amdgcn_udot4(rows[x][1], rows[x][1], e_half, false);
        }
        double A[4][8];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y) A[x][y] = 0.0;
#pragma unroll 1
        for (int w = 0; w * kDctWin < r_hi; ++w) {
            __builtin_amdgcn_wave_barrier();
            if (w == 0) dct_fwd_window<0>(pix, lds, lane, std::make_index_sequence<8>{});
            else dct_fwd_window<1>(pix, lds, lane, std::make_index_sequence<8>{});
            __builtin_amdgcn_wave_barrier();
            const int j0 = w * kDctWin, j1 = min(r_hi, j0 + kDctWin);
            for (int j = j0; j < j1; ++j) {
                const double b = lds[(j - j0) * 64 + lane];
                const DctStep &E = S[j];                     // wave-uniform: scalar loads
                double u[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) u[x] = b * E.ck[4 * h + x];
#pragma unroll
                for (int y = 0; y < 8; ++y) {
                    const double cl = E.cl[y];
#pragma unroll
                    for (int x = 0; x < 4; ++x) A[x][y] = fma(u[x], cl, A[x][y]);
                }
                uint32_t sq = e_half, cross = 0;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    int q[8];
#pragma unroll
                    for (int y = 0; y < 8; ++y)
                        q[y] = min(max(__double2loint(A[x][y] + 6755399441055744.0), 0), 255);
                    score_row(q, rows[x][0], rows[x][1], sq, cross);
                }
                unsigned err = sq - 2u * cross;
                if (j + 1 >= r_lo) {
                    err = wave_add(active ? err : 0u);
                    if (lane == 0 && err) atomicAdd(out + (j + 1 - r_lo), (unsigned long long)err);
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- kernels

struct TileRef {
    int image;
    bool active;
    uint32_t pix[8][2];
};

// locate the image of a tile (binary search over the tiles' start indices) and
// load the lane's 8x8 block
__device__ __forceinline__ void load_tile(const BatchArgs &a, int tile, int lane, TileRef &t) {
    int lo = 0, hi = a.n_images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.img[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
    }
    t.image = lo;
    const BatchImg &I = a.img[lo];
    const int b = (tile - I.tile_start) * 64 + lane;
    t.active = b < I.nblocks;
    const int bb = t.active ? b : 0;
    const int by = bb / I.nbx, bx = bb - by * I.nbx;
    const uint8_t *src = a.base + I.offset + int64_t(8 * by) * I.pitch + 8 * bx;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const u32x2 v = *(const u32x2 *)(src + int64_t(x) * I.pitch);
        t.pix[x][0] = v.x;
        t.pix[x][1] = v.y;
    }
}

// integer transforms: items are (tile, group) with group g taking the integer
// transforms g, g + split, ... of the list
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch_int(const BatchArgs a) {
    const int lane = threadIdx.x;
    const int items = a.total_tiles * a.split;
    const int nr = a.r_hi - a.r_lo + 1;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tile = it / a.split, grp = it - tile * a.split;
        TileRef T;
        load_tile(a, tile, lane, T);
        for (int ii = grp; ii < a.n_int; ii += a.split) {
            const int ti = a.int_pos[ii];
            unsigned long long *out = a.sse + (int64_t(T.image) * a.n_transforms + ti) * nr;
            switch (a.tids[ti]) {
                case ADCT_T1: sweep_int<ADCT_T1>(T.pix, T.active, out, a.r_lo, a.r_hi, lane); break;
                case ADCT_T2: sweep_int<ADCT_T2>(T.pix, T.active, out, a.r_lo, a.r_hi, lane); break;
                case ADCT_LO: sweep_int<ADCT_LO>(T.pix, T.active, out, a.r_lo, a.r_hi, lane); break;
                case ADCT_T6: sweep_int<ADCT_T6>(T.pix, T.active, out, a.r_lo, a.r_hi, lane); break;
                case ADCT_RDCT: sweep_int<ADCT_RDCT>(T.pix, T.active, out, a.r_lo, a.r_hi, lane); break;
                default: sweep_int<ADCT_T4>(T.pix, T.active, out, a.r_lo, a.r_hi, lane); break;
            }
        }
    }
}

// the exact DCT: items are (tile, DCT entry of the list)
__global__ __launch_bounds__(64) void k_batch_dct(const BatchArgs a) {
    const int lane = threadIdx.x;
    const int items = a.total_tiles * a.n_dct;
    const int nr = a.r_hi - a.r_lo + 1;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tile = it / a.n_dct, d = it - tile * a.n_dct;
        TileRef T;
        load_tile(a, tile, lane, T);
        unsigned long long *out = a.sse + (int64_t(T.image) * a.n_transforms + a.dct_pos[d]) * nr;
        sweep_dct(T.pix, T.active, out, a.r_lo, a.r_hi, lane);
    }
}

__global__ void k_zero(unsigned long long *p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

int device_cus() {
    static thread_local int cached_dev = -1, cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != cached_dev) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cached_dev = dev;
    }
    return cus;
}

// zero fill, then the DCT kernel (if the list has the DCT), then the integer
// kernel (if it has integer transforms).  wgs_per_cu sets the integer kernel's
// resident single-wave workgroups per compute unit; the DCT kernel fills every
// slot its 32 KB of LDS allows.
adct_status enqueue(const BatchArgs &a, int wgs_per_cu, hipStream_t s) {
    const int64_t n = int64_t(a.n_images) * a.n_transforms * (a.r_hi - a.r_lo + 1);
    hipLaunchKernelGGL(k_zero, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a.sse, n);
    ADCT_HIP(hipGetLastError());
    const int cus = device_cus();
    if (cus <= 0) return fail(ADCT_EDEVICE, "cannot query the device");
    if (a.n_dct > 0) {
        int per_cu = 0;
        ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_dct, 64, 0));
        if (per_cu < 1) per_cu = 1;
        const int64_t items = int64_t(a.total_tiles) * a.n_dct;
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(items, int64_t(per_cu) * cus)));
        hipLaunchKernelGGL(k_batch_dct, dim3(grid), dim3(64), 0, s, a);
        ADCT_HIP(hipGetLastError());
    }
    if (a.n_int > 0) {
        const int64_t items = int64_t(a.total_tiles) * a.split;
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(items, int64_t(wgs_per_cu) * cus)));
        hipLaunchKernelGGL(k_batch_int, dim3(grid), dim3(64), 0, s, a);
        ADCT_HIP(hipGetLastError());
    }
    return ADCT_OK;
}

}  // namespace
}  // namespace adct

using namespace adct;

struct adct_batch_plan_s {
    BatchArgs args;
    int wgs_per_cu = 4;
    double tuned_ms = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

adct_status build_args(const uint8_t *base, const adct_plane *images, int n_images,
                       const adct_transform_id *transforms, int n_transforms, int r_lo, int r_hi,
                       uint64_t *sse, BatchArgs *a) {
    if (!base || !images || !transforms || !sse) return fail(ADCT_EINVAL, "null argument");
    if (n_images < 1 || n_images > kMaxBatchImages)
        return fail(ADCT_ERANGE, "n_images must be in [1, 64] per launch");
    if (n_transforms < 1 || n_transforms > kMaxBatchTransforms)
        return fail(ADCT_ERANGE, "n_transforms must be in [1, 8]");
    if (r_lo < 1 || r_hi > 64 || r_lo > r_hi) return fail(ADCT_ERANGE, "need 1 <= r_lo <= r_hi <= 64");
    if ((reinterpret_cast<uintptr_t>(base) & 7) || (reinterpret_cast<uintptr_t>(sse) & 7))
        return fail(ADCT_EDIM, "base and sse must be 8-byte aligned");
    memset(a, 0, sizeof(*a));
    a->base = base;
    a->sse = reinterpret_cast<unsigned long long *>(sse);
    a->n_images = n_images;
    a->n_transforms = n_transforms;
    a->r_lo = r_lo;
    a->r_hi = r_hi;
    a->split = 1;
    for (int t = 0; t < n_transforms; ++t) {
        const int id = transforms[t];
        if (id < ADCT_DCT || id > ADCT_T4) return fail(ADCT_EINVAL, "unknown or custom transform in a batch");
        a->tids[t] = id;
        if (id == ADCT_DCT) a->dct_pos[a->n_dct++] = t;
        else a->int_pos[a->n_int++] = t;
    }
    int tiles = 0;
    for (int i = 0; i < n_images; ++i) {
        const adct_plane &p = images[i];
        if (p.H <= 0 || p.W <= 0 || (p.H & 7) || (p.W & 7) || p.pitch < p.W || (p.pitch & 7) || (p.offset & 7))
            return fail(ADCT_EDIM, "image " + std::to_string(i) +
                                       ": H, W multiples of 8, pitch >= W, pitch and offset multiples of 8");
        BatchImg &d = a->img[i];
        d.offset = p.offset;
        d.pitch = p.pitch;
        d.nbx = p.W / 8;
        d.nblocks = (p.H / 8) * (p.W / 8);
        d.tile_start = tiles;
        tiles += (d.nblocks + 63) / 64;
    }
    a->total_tiles = tiles;
    return ADCT_OK;
}

}  // namespace

extern "C" {

adct_status adct_evaluate_batch(const uint8_t *base, const adct_plane *images, int n_images,
                                const adct_transform_id *transforms, int n_transforms, int r_lo,
                                int r_hi, uint64_t *sse, int wgs_per_cu, int split,
                                adct_stream_t stream) {
    BatchArgs a;
    adct_status st = build_args(base, images, n_images, transforms, n_transforms, r_lo, r_hi, sse, &a);
    if (st) return st;
    if (wgs_per_cu < 1 || wgs_per_cu > 16) return fail(ADCT_ERANGE, "wgs_per_cu must be in [1, 16]");
    if (split < 1 || split > n_transforms) return fail(ADCT_ERANGE, "split must be in [1, n_transforms]");
    a.split = std::min(split, std::max(a.n_int, 1));
    return enqueue(a, wgs_per_cu, reinterpret_cast<hipStream_t>(stream));
}

adct_status adct_batch_plan_create(const uint8_t *base, const adct_plane *images, int n_images,
                                   const adct_transform_id *transforms, int n_transforms, int r_lo,
                                   int r_hi, uint64_t *sse, int autotune, adct_batch_plan *out,
                                   adct_stream_t stream) {
    if (!out) return fail(ADCT_EINVAL, "out is null");
    *out = nullptr;
    adct_batch_plan p = new adct_batch_plan_s();
    adct_status st = build_args(base, images, n_images, transforms, n_transforms, r_lo, r_hi, sse, &p->args);
    if (st) {
        delete p;
        return st;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (autotune) {
        // time every (workgroups per CU, transform split) candidate on the real
        // input and keep the fastest
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            delete p;
            return fail(ADCT_EDEVICE, "hipEventCreate failed");
        }
        double best = 1e30;
        int best_w = 4, best_s = 1;
        const int n_split = std::max(p->args.n_int, 1);
        for (int split = 1; split <= n_split; ++split) {
            if (n_split % split) continue;
            for (int w : {4, 6, 8, 12, 16}) {
                BatchArgs a = p->args;
                a.split = split;
                st = enqueue(a, w, s);                         // warm
                if (!st) st = hipEventRecord(e0, s) == hipSuccess ? ADCT_OK : ADCT_EDEVICE;
                if (!st) st = enqueue(a, w, s);
                if (!st) st = hipEventRecord(e1, s) == hipSuccess ? ADCT_OK : ADCT_EDEVICE;
                float ms = 0.f;
                if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    st = fail(ADCT_EDEVICE, "timing failed");
                if (st) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    delete p;
                    return st;
                }
                if (ms < best) {
                    best = ms;
                    best_w = w;
                    best_s = split;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        p->wgs_per_cu = best_w;
        p->args.split = best_s;
        p->tuned_ms = best;
    }
    // capture zero-fill + sweep into a graph on a private stream
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return fail(ADCT_EDEVICE, "hipStreamCreate failed");
    }
    st = ADCT_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        st = fail(ADCT_EDEVICE, "hipStreamBeginCapture failed");
    if (!st) {
        const adct_status st2 = enqueue(p->args, p->wgs_per_cu, cap);
        const hipError_t e = hipStreamEndCapture(cap, &p->graph);
        if (st2) st = st2;
        else if (e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
    }
    if (!st) {
        const hipError_t e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
    }
    (void)hipStreamDestroy(cap);
    if (st) {
        if (p->graph) (void)hipGraphDestroy(p->graph);
        delete p;
        return st;
    }
    *out = p;
    return ADCT_OK;
}

adct_status adct_batch_plan_launch(adct_batch_plan plan, adct_stream_t stream) {
    if (!plan) return fail(ADCT_EINVAL, "plan is null");
    ADCT_HIP(hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream)));
    return ADCT_OK;
}

adct_status adct_batch_plan_info(adct_batch_plan plan, int *wgs_per_cu, int *split, double *tuned_ms) {
    if (!plan) return fail(ADCT_EINVAL, "plan is null");
    if (wgs_per_cu) *wgs_per_cu = plan->wgs_per_cu;
    if (split) *split = plan->args.split;
    if (tuned_ms) *tuned_ms = plan->tuned_ms;
    return ADCT_OK;
}

adct_status adct_batch_plan_destroy(adct_batch_plan plan) {
    if (!plan) return ADCT_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return ADCT_OK;
}

}  // extern "C"
