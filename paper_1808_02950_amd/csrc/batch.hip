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
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "adct_internal.hpp"
#include "wave.hpp"

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
    unsigned *ctr;                    // [2] work counters (integer, DCT) or null: grid stride
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

// As score_row for a row of rounded values that still need clipping to
// [0, 255] (|q| < 2^15): pairs as int16 halves, one saturating pack per pair.
__device__ __forceinline__ void score_row_sat(const int (&q)[8], uint32_t w0, uint32_t w1, uint32_t &sq,
                                              uint32_t &cross) {
    uint32_t b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        b[i] = sat_pk_u8_i16(__builtin_amdgcn_perm(uint32_t(q[2 * i + 1]), uint32_t(q[2 * i]), 0x05040100u));
    const uint32_t lo = b[0] | (b[1] << 16);
    const uint32_t hi = b[2] | (b[3] << 16);
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

// (every lane of the wave is active where it is called)
__device__ __forceinline__ unsigned wave_add(unsigned v) { return wave_sum_u32(v); }

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

// Exact round-half-to-even(n / L) without a 32-bit multiply or a clip.  The
// sweep keeps P = n + L/2, so the half-up quotient is q = floor(P / L), found
// in float: write L = 2^s d (s = 0 for small L, else the power of two of L, so
// d is odd); floor(P / L) = floor(v / d) for v = P >> s, whose fractions are
// multiples of 1/d, and fma(v, 1/d, 1/(2d)) = (v + 1/2) fl(1/d) rounded lies
// within (257.5 * 2^-24 + 2^-16) < 1/(2d) of v/d + 1/(2d) while v/d <= 257,
// so truncating it gives q.  Above that the float is still monotone in P and
// every such q saturates to 255; for P < 0 the truncation is at most 0, which
// saturates to 0.  At a tie P = L q exactly: the remainder x = P - L q is zero
// there and in [1, L) elsewhere (a wrong q below 0 or above 256 makes x
// negative or at least L, and leaves no tie to fix), so min(x, 1) is 0 exactly
// at a tie, where an odd q loses its low bit.  The result, in [-2042, 2042],
// is clipped by the saturating byte pack of score_row_sat.
template <int ID>
struct IntRound {
    static constexpr int32_t L = Tf<ID>::L();
    static constexpr int32_t v2() {
        int32_t s = 0;
        while ((L >> s & 1) == 0) ++s;
        return s;
    }
    static constexpr int32_t kS = L >= 4096 ? v2() : 0;
    static constexpr int32_t kD = L >> kS;               // divisor of the float quotient
    static_assert(kD < 16000, "divisor too large for the float quotient");
    static_assert(L % 2 == 0, "the sweep adds L/2");
};

// wave-uniform constant of the rounding, held in a scalar register (a VOP3
// instruction takes no 32-bit literal on this target)
struct IntRoundRegs {
    int32_t mL;           // -L
};

template <int ID>
__device__ __forceinline__ IntRoundRegs int_round_regs() {
    IntRoundRegs r;
    asm("s_mov_b32 %0, %1" : "=s"(r.mL) : "i"(-IntRound<ID>::L));
    return r;
}

// P = n + L/2 -> round-half-to-even(n / L), unclipped
template <int ID>
__device__ __forceinline__ int rne_int(int P, const IntRoundRegs &c) {
    using R = IntRound<ID>;
    constexpr float kInv = 1.0f / float(R::kD);
    constexpr float kOff = 0.5f / float(R::kD);
    const float f = __builtin_fmaf(float(R::kS ? (P >> R::kS) : P), kInv, kOff);
    const int q = int(f);
    const uint32_t x = uint32_t(__mul24(q, c.mL) + P);
    // min(x, 1) as one instruction (left to itself the compiler turns the
    // comparison with zero into a compare and a select)
    uint32_t m;
    asm("v_min_u32 %0, 1, %1" : "=v"(m) : "v"(x));
    return q & int(m | ~1u);
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
    int A[8][8];      // n + L/2: the reconstruction numerator, biased for rne_int
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) A[x][y] = IntRound<ID>::L / 2;
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
            for (int y = 0; y < 8; ++y) q[y] = rne_int<ID>(A[x][y], rc);
            score_row_sat(q, pix[x][0], pix[x][1], sq, cross);
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

// The item a single-wave workgroup takes after `it`: the next one of its grid
// stride, or, with a work counter, the next one nobody has taken (workgroup b
// starts with item b, so the counter numbers the items from gridDim.x on).
// The counter balances the two kernels when they share the chip: a workgroup
// that becomes resident late takes only what is left.
__device__ __forceinline__ int next_item(unsigned *ctr, int it) {
    if (!ctr) return it + int(gridDim.x);
    unsigned v = 0;
    if (threadIdx.x == 0) v = atomicAdd(ctr, 1u);
    return int(gridDim.x) + __builtin_amdgcn_readfirstlane(int(__builtin_amdgcn_readlane(int(v), 0)));
}

// integer transforms: items are (tile, group) with group g taking the integer
// transforms g, g + split, ... of the list
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch_int(const BatchArgs a) {
    const int lane = threadIdx.x;
    const int items = a.total_tiles * a.split;
    const int nr = a.r_hi - a.r_lo + 1;
    unsigned *ctr = a.ctr ? a.ctr + 0 : nullptr;
    for (int it = blockIdx.x; it < items; it = next_item(ctr, it)) {
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
    unsigned *ctr = a.ctr ? a.ctr + 1 : nullptr;
    for (int it = blockIdx.x; it < items; it = next_item(ctr, it)) {
        const int tile = it / a.n_dct, d = it - tile * a.n_dct;
        TileRef T;
        load_tile(a, tile, lane, T);
        unsigned long long *out = a.sse + (int64_t(T.image) * a.n_transforms + a.dct_pos[d]) * nr;
        sweep_dct(T.pix, T.active, out, a.r_lo, a.r_hi, lane);
    }
}

__global__ void k_zero(unsigned long long *p, int64_t n, unsigned *ctr) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
    if (ctr && i < 2) ctr[i] = 0u;
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
// slot its LDS and registers allow, or at most dct_per_cu per CU if that is set.  With a second stream s2 (and two events) the
// DCT kernel runs on s2 beside the integer kernel: s2 waits for the zero fill,
// s waits for the DCT kernel before it returns (a fork and a join, which stream
// capture records as two graph branches).
adct_status enqueue(const BatchArgs &a, int wgs_per_cu, hipStream_t s, hipStream_t s2 = nullptr,
                    hipEvent_t fork = nullptr, hipEvent_t join = nullptr, int dct_per_cu = 0) {
    const int64_t n = int64_t(a.n_images) * a.n_transforms * (a.r_hi - a.r_lo + 1);
    hipLaunchKernelGGL(k_zero, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a.sse, n, a.ctr);
    ADCT_HIP(hipGetLastError());
    const int cus = device_cus();
    if (cus <= 0) return fail(ADCT_EDEVICE, "cannot query the device");
    const bool branches = s2 && fork && join && a.n_dct > 0 && a.n_int > 0;
    hipStream_t sd = s;
    if (branches) {
        ADCT_HIP(hipEventRecord(fork, s));
        ADCT_HIP(hipStreamWaitEvent(s2, fork, 0));
        sd = s2;
    }
    if (a.n_dct > 0) {
        int per_cu = 0;
        ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_dct, 64, 0));
        if (per_cu < 1) per_cu = 1;
        if (dct_per_cu > 0) per_cu = std::min(per_cu, dct_per_cu);
        const int64_t items = int64_t(a.total_tiles) * a.n_dct;
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(items, int64_t(per_cu) * cus)));
        hipLaunchKernelGGL(k_batch_dct, dim3(grid), dim3(64), 0, sd, a);
        ADCT_HIP(hipGetLastError());
    }
    if (a.n_int > 0) {
        const int64_t items = int64_t(a.total_tiles) * a.split;
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(items, int64_t(wgs_per_cu) * cus)));
        hipLaunchKernelGGL(k_batch_int, dim3(grid), dim3(64), 0, s, a);
        ADCT_HIP(hipGetLastError());
    }
    if (branches) {
        ADCT_HIP(hipEventRecord(join, s2));
        ADCT_HIP(hipStreamWaitEvent(s, join, 0));
    }
    return ADCT_OK;
}

// a second stream (default priority) and the fork / join events of a plan
struct Branch {
    hipStream_t s2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    adct_status make() {
        ADCT_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        ADCT_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        ADCT_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        return ADCT_OK;
    }
    ~Branch() {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (s2) (void)hipStreamDestroy(s2);
    }
};

}  // namespace
}  // namespace adct

using namespace adct;

// A plan is the argument block, its tuned schedule, the two work counters and
// the second stream with its fork / join events.  Launching enqueues the
// schedule; the mutex keeps two host threads from interleaving the event
// records of one plan.
struct adct_batch_plan_s {
    BatchArgs args;
    int wgs_per_cu = 4;
    int dct_per_cu = 0;
    double tuned_ms = 0.0;
    Branch br;
    std::mutex mu;
    ~adct_batch_plan_s() {
        if (args.ctr) (void)hipFree(args.ctr);
    }
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
    Branch &br = p->br;
    if (adct_status stb = br.make()) {
        delete p;
        return stb;
    }
    if (hipMalloc(&p->args.ctr, 2 * sizeof(unsigned)) != hipSuccess) {
        p->args.ctr = nullptr;
        delete p;
        return fail(ADCT_EDEVICE, "cannot allocate the work counters");
    }
    if (autotune) {
        // time every (workgroups per CU, transform split) candidate on the real
        // input and keep the fastest
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            delete p;
            return fail(ADCT_EDEVICE, "hipEventCreate failed");
        }
        double best = 1e30;
        int best_w = 4, best_s = 1, best_d = 0;
        const int n_split = std::max(p->args.n_int, 1);
        const bool both = p->args.n_int > 0 && p->args.n_dct > 0;
        for (int split = 1; split <= n_split; ++split) {
            if (n_split % split) continue;
            for (int w : {4, 6, 8, 12, 16})
            for (int d : {0, 4, 2}) {
                if (d && !both) continue;
                BatchArgs a = p->args;
                a.split = split;
                st = enqueue(a, w, s, br.s2, br.fork, br.join, d);     // warm
                if (!st) st = hipEventRecord(e0, s) == hipSuccess ? ADCT_OK : ADCT_EDEVICE;
                if (!st) st = enqueue(a, w, s, br.s2, br.fork, br.join, d);
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
                    best_d = d;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        p->wgs_per_cu = best_w;
        p->dct_per_cu = best_d;
        p->args.split = best_s;
        p->tuned_ms = best;
    }
    *out = p;
    return ADCT_OK;
}
adct_status adct_batch_plan_launch(adct_batch_plan plan, adct_stream_t stream) {
    if (!plan) return fail(ADCT_EINVAL, "plan is null");
    std::lock_guard<std::mutex> lock(plan->mu);
    return enqueue(plan->args, plan->wgs_per_cu, reinterpret_cast<hipStream_t>(stream), plan->br.s2,
                   plan->br.fork, plan->br.join, plan->dct_per_cu);
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
    // the plan's kernels may still run on its second stream
    (void)hipStreamSynchronize(plan->br.s2);
    delete plan;
    return ADCT_OK;
}

}  // extern "C"
