// Internal definitions shared by the library's translation units (not the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <numeric>
#include <string>

#include "adct.h"

namespace adct {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
adct_status fail(adct_status s, const std::string &msg);
adct_status hip_fail(hipError_t e, const char *what);

#define ADCT_HIP(call)                                                 \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::adct::hip_fail(e_, #call);      \
    } while (0)

// ---------------------------------------------------------------- matrices
//
// The library's own copy of the integer matrices (T LO stored doubled so it is
// integral; the scale S is invariant to a positive factor).  T1 and T2 are the
// matrices the paper derives (Sec. 4.1); RDCT, LO, T6, T4 are from its table of
// common low-complexity matrices (Sec. 2).

struct Mat8 {
    int8_t m[8][8];
};

constexpr Mat8 kT1 = {{{1, 1, 1, 1, 1, 1, 1, 1},
                       {2, 2, 1, 0, 0, -1, -2, -2},
                       {2, 1, -1, -2, -2, -1, 1, 2},
                       {1, 0, -2, -2, 2, 2, 0, -1},
                       {1, -1, -1, 1, 1, -1, -1, 1},
                       {2, -2, 0, 1, -1, 0, 2, -2},
                       {1, -2, 2, -1, -1, 2, -2, 1},
                       {0, -1, 2, -2, 2, -2, 1, 0}}};

constexpr Mat8 kT2 = {{{1, 1, 1, 1, 1, 1, 1, 1},
                       {2, 1, 2, 0, 0, -2, -1, -2},
                       {2, 1, -1, -2, -2, -1, 1, 2},
                       {2, 0, -2, -1, 1, 2, 0, -2},
                       {1, -1, -1, 1, 1, -1, -1, 1},
                       {1, -2, 0, 2, -2, 0, 2, -1},
                       {1, -2, 2, -1, -1, 2, -2, 1},
                       {0, -2, 1, -2, 2, -1, 2, 0}}};

constexpr Mat8 kLOx2 = {{{2, 2, 2, 2, 2, 2, 2, 2},
                         {2, 2, 2, 0, 0, -2, -2, -2},
                         {2, 1, -1, -2, -2, -1, 1, 2},
                         {2, 0, -2, -2, 2, 2, 0, -2},
                         {2, -2, -2, 2, 2, -2, -2, 2},
                         {2, -2, 0, 2, -2, 0, 2, -2},
                         {1, -2, 2, -1, -1, 2, -2, 1},
                         {0, -2, 2, -2, 2, -2, 2, 0}}};

constexpr Mat8 kT6 = {{{1, 1, 1, 1, 1, 1, 1, 1},
                       {2, 1, 1, 0, 0, -1, -1, -2},
                       {2, 1, -1, -2, -2, -1, 1, 2},
                       {1, 0, -2, -1, 1, 2, 0, -1},
                       {1, -1, -1, 1, 1, -1, -1, 1},
                       {1, -2, 0, 1, -1, 0, 2, -1},
                       {1, -2, 2, -1, -1, 2, -2, 1},
                       {0, -1, 1, -2, 2, -1, 1, 0}}};

constexpr Mat8 kRDCT = {{{1, 1, 1, 1, 1, 1, 1, 1},
                         {1, 1, 1, 0, 0, -1, -1, -1},
                         {1, 0, 0, -1, -1, 0, 0, 1},
                         {1, 0, -1, -1, 1, 1, 0, -1},
                         {1, -1, -1, 1, 1, -1, -1, 1},
                         {1, -1, 0, 1, -1, 0, 1, -1},
                         {0, -1, 1, 0, 0, 1, -1, 0},
                         {0, -1, 1, -1, 1, -1, 1, 0}}};

constexpr Mat8 kT4 = {{{1, 1, 1, 1, 1, 1, 1, 1},
                       {1, 1, 1, 0, 0, -1, -1, -1},
                       {1, 1, -1, -1, -1, -1, 1, 1},
                       {1, 0, -1, -1, 1, 1, 0, -1},
                       {1, -1, -1, 1, 1, -1, -1, 1},
                       {1, -1, 0, 1, -1, 0, 1, -1},
                       {1, -1, 1, -1, -1, 1, -1, 1},
                       {0, -1, 1, -1, 1, -1, 1, 0}}};

constexpr const Mat8 &builtin(int id) {
    return id == ADCT_T1 ? kT1 : id == ADCT_T2 ? kT2 : id == ADCT_LO ? kLOx2
         : id == ADCT_T6 ? kT6 : id == ADCT_RDCT ? kRDCT : kT4;
}

// JPEG zig-zag: kZZ[z] = 8*row + col of the z-th scanned coefficient.
constexpr int kZZ[64] = {
    0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,
    12, 19, 26, 33, 40, 48, 41, 34, 27, 20, 13, 6,  7,  14, 21, 28,
    35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51,
    58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

struct ZZInv {
    int pos[64];   // pos[8 * row + col] = zig-zag position
};
constexpr ZZInv make_zz_inv() {
    ZZInv t{};
    for (int z = 0; z < 64; ++z) t.pos[kZZ[z]] = z;
    return t;
}
constexpr ZZInv kZZInv = make_zz_inv();
constexpr int zz_pos(int k, int l) { return kZZInv.pos[8 * k + l]; }

// 1/sqrt(v) in float64 from Newton's iteration for sqrt(v): the same value in
// the compile-time tables of the built-in matrices and in the run-time tables
// the host builds for a caller's matrix.
constexpr double inv_sqrt_newton(int64_t v) {
    double r = double(v);
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + double(v) / r);
    return 1.0 / r;
}

// Scale classes: the distinct values of n_k n_l of a matrix, numbered in
// increasing order (at most 36 for 8 distinct row norms).  The quantiser
// constants are per class, so a kernel holds one copy of each.
constexpr int kMaxClasses = 36;

// class index of n_k n_l among the distinct products of n (ascending)
constexpr int class_of(const int32_t (&n)[8], int k, int l) {
    const int64_t v = int64_t(n[k]) * n[l];
    int below = 0;
    for (int a = 0; a < 64; ++a) {
        const int64_t u = int64_t(n[a >> 3]) * n[a & 7];
        if (u >= v) continue;
        bool first = true;                     // count each distinct smaller value once
        for (int c = 0; c < a && first; ++c)
            if (int64_t(n[c >> 3]) * n[c & 7] == u) first = false;
        below += first ? 1 : 0;
    }
    return below;
}

// Per-transform constants derived at compile time.
template <int ID>
struct Tf {
    static constexpr const Mat8 &M = builtin(ID);
    static constexpr int8_t t(int k, int m) { return M.m[k][m]; }
    static constexpr int32_t n(int k) {
        int32_t s = 0;
        for (int m = 0; m < 8; ++m) s += int32_t(M.m[k][m]) * M.m[k][m];
        return s;
    }
    static constexpr int32_t L1() {
        int32_t l = 1;
        for (int k = 0; k < 8; ++k) l = std::lcm(l, n(k));
        return l;
    }
    // c_k = L1 / n_k as a table, so that a use with an unrolled index folds to a
    // constant instead of running the lcm loops on the device
    struct CTab {
        int32_t c[8];
    };
    static constexpr CTab make_c() {
        CTab t{};
        for (int k = 0; k < 8; ++k) t.c[k] = L1() / n(k);
        return t;
    }
    static constexpr CTab kC = make_c();
    static constexpr int32_t c(int k) { return kC.c[k]; }
    struct Tables {
        int32_t mu[64];   // mu with mu^2 = n_k n_l, or 0 when n_k n_l is not a square
        double skl[64];   // s_k s_l = 1 / sqrt(n_k n_l)
    };
    static constexpr Tables make_tables() {
        Tables t{};
        for (int k = 0; k < 8; ++k)
            for (int l = 0; l < 8; ++l) {
                const int32_t v = n(k) * n(l);
                int32_t m = 0;
                for (int32_t c = 1; c * c <= v; ++c)
                    if (c * c == v) m = c;
                t.mu[8 * k + l] = m;
                t.skl[8 * k + l] = inv_sqrt_newton(v);
            }
        return t;
    }
    static constexpr Tables kTab = make_tables();
    static constexpr int32_t mu(int k, int l) { return kTab.mu[8 * k + l]; }
    struct NTab {
        int32_t n[8];
    };
    static constexpr NTab make_n() {
        NTab t{};
        for (int k = 0; k < 8; ++k) t.n[k] = n(k);
        return t;
    }
    static constexpr NTab kN = make_n();
    struct ClsTab {
        int32_t c[64];
    };
    static constexpr ClsTab make_cls() {
        ClsTab t{};
        for (int i = 0; i < 64; ++i) t.c[i] = class_of(kN.n, i >> 3, i & 7);
        return t;
    }
    static constexpr ClsTab kCls = make_cls();
    // scale class of (k, l), a table filled at compile time
    static constexpr int cls(int k, int l) { return kCls.c[8 * k + l]; }
    static constexpr double skl(int k, int l) { return kTab.skl[8 * k + l]; }
    static constexpr int32_t L() { return L1() * L1(); }
    // |Y| fits int16 for 8-bit input (checked by the host bound routine too).
    static constexpr bool kSymmetric() {
        for (int k = 0; k < 8; ++k)
            for (int m = 0; m < 4; ++m)
                if (M.m[k][7 - m] != ((k & 1) ? -M.m[k][m] : M.m[k][m])) return false;
        return true;
    }
    static_assert(kSymmetric(), "even rows symmetric, odd rows antisymmetric");
};

// ---------------------------------------------------------------- launch args

constexpr int kMaxPlanes = 4;

struct PlaneArg {
    int64_t in_off;     // byte offset of the plane inside a frame (input)
    int64_t out_off;    // byte offset inside an output frame
    int32_t pitch_in;
    int32_t pitch_out;
    int32_t nbx;        // blocks per block-row
    int32_t nblocks;    // blocks in the plane
    int32_t wave_start; // first wave of this plane inside a frame
    int32_t block_off;  // first block of this plane inside a frame
    uint32_t nbx_m;     // n / nbx = umulhi(n, nbx_m) >> nbx_s for 0 <= n < 2^31
    int32_t nbx_s;      //   (nbx_s < 0: nbx == 1)
};

// Two int16 halves of x saturated to [0, 255] and packed as bytes 0 and 1 (the
// upper half of the result is zero).
__device__ __forceinline__ uint32_t sat_pk_u8_i16(uint32_t x) {
    uint32_t r;
    asm("v_sat_pk_u8_i16 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Exact division of 0 <= n < 2^31 by a wave-uniform divisor d through a
// multiply-high and a shift (Granlund-Montgomery with a 32-bit multiplier):
// with l = ceil(log2 d), m = ceil(2^(31 + l) / d) < 2^32 and n / d =
// (n m) >> (31 + l).  Filled on the host (magic_u31), used by the tile walks.
inline void magic_u31(uint32_t d, uint32_t *m, int32_t *s) {
    if (d <= 1) {
        *m = 0;
        *s = -1;
        return;
    }
    int l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    *m = uint32_t(((uint64_t(1) << (31 + l)) + d - 1) / d);
    *s = l - 1;
}

struct CodecArgs {
    const uint8_t *in;
    uint8_t *out;
    int16_t *coef;
    float *coef_f;
    unsigned long long *sse;
    int64_t fs_in;      // frame stride of `in` (bytes)
    int64_t fs_out;     // frame stride of `out`
    int32_t n_frames;
    int32_t n_planes;
    int32_t waves_per_frame;
    int32_t blocks_per_frame;
    int32_t r;
    int32_t pad;
    PlaneArg pl[kMaxPlanes];
    int32_t step;        // quantiser step (0: zonal coding only)
    float inv_step_f;    // 1 / step
    double inv_step_d;   // 1 / step
    double step_d;       // step
    uint32_t wpf_m;      // division by waves_per_frame (see magic_u31)
    int32_t wpf_s;
};

// Quantiser constants of the built-in codec kernels per scale class (a second
// kernel argument; zero when there is no quantiser), with d = step mu for a
// class n_k n_l = mu^2.
struct QuantTables {
    float qc1[kMaxClasses];       // 1 / d                       (rational classes)
    float qc2[kMaxClasses];       // (d + 1/2) / (2 d)           (rational classes)
    double qinv[kMaxClasses];     // s_k s_l / step              (irrational classes)
    double qdeq[kMaxClasses];     // step s_k s_l: dequantised B = q qdeq
};

struct DctArgs {
    const uint8_t *in;
    uint8_t *out;
    float *coef_f;       // B (float32), [block][r]
    int16_t *coef_q;     // quantised levels, [block][r] (step > 0)
    unsigned long long *sse;
    int64_t fs_in;
    int64_t fs_out;
    int32_t n_frames;
    int32_t n_planes;
    int32_t waves_per_frame;
    int32_t blocks_per_frame;
    int32_t r;
    int32_t step;
    float inv_step;
    int32_t wpf_s;             // division by waves_per_frame (see magic_u31)
    uint32_t wpf_m;
    int32_t pad;
    PlaneArg pl[kMaxPlanes];   // wave_start counts 16-block tiles
    float C[64];               // orthonormal DCT-II, C[8k + x]
};

// kProbe: the loads and stores of kEvaluate without its arithmetic (the
// achievable HBM rate of the codec's read / write mix).
enum Mode { kEncode = 0, kDecode = 1, kEvaluate = 2, kProbe = 3 };

// Constants of an integer matrix given at run time (ADCT_CUSTOM, and the
// float-coefficient decode of the built-in matrices), a second kernel argument
// of the run-time codec kernels.  All entries are wave-uniform.
// Exact rounding of dequantised reconstructions that can sit on a half (a step
// for which step / mu has an even reduced denominator for some class with
// n_k n_l = mu^2).  Write n_k n_l = mu^2 r with r squarefree: 1 / sqrt(n_k n_l)
// = w sqrt(r) / D with D = lcm(mu r) and w = D / (mu r), so a pixel is
//   (step / D) (N_0 + N_1 sqrt(p) + N_2 sqrt(q) + N_3 sqrt(r3)),
// N_c the sum over the coefficients of class c of C_kl T[k][x] T[l][y] w_kl,
// where the generators p, q give every r that occurs (r3 the squarefree part
// of p q, sqrt(p q) = g sqrt(r3)).  The kernel decides a pixel within tol of a
// half by the exact sign of the difference in that field.
struct RtSettle {
    int32_t on;          // nonzero: decide pixels near a half exactly
    int32_t p, q, g;     // generators (1 when absent), sqrt(p q) = g sqrt(r3)
    int64_t D;
    double tol_c;        // tolerance per unit of sum |C_kl| s_k s_l (float64 error bound)
    int32_t w[64];       // w_kl
    int8_t cls[64];      // 0: rational, 1: sqrt p, 2: sqrt q, 3: sqrt r3
};

struct RtMatArgs {
    int32_t t[64];       // T[k][m] at 8k + m
    int32_t mu[64];      // mu with mu^2 = n_k n_l, 0 when n_k n_l is not a square
    float inv_2mu[64];   // 0.5 / mu (rational classes)
    int64_t ckl[64];     // c_k c_l with c_k = L1 / n_k, L1 = lcm(n): exact inverse weights
    double skl[64];      // s_k s_l = 1 / sqrt(n_k n_l)
    int64_t L;           // L1^2, the exact inverse's denominator
    double inv_2L;       // 1 / (2 L)
    RtSettle st;
};

// Bounds of the exact near-half decision (checked on the host): every field
// component below 2^52 in magnitude, p q <= 1024, so the second-level values
// stay inside 128-bit words and their squares inside 256 bits.
constexpr int64_t kSettleMaxComp = int64_t(1) << 52;
constexpr int32_t kSettleMaxPQ = 1024;

// Word sizes the run-time kernels assume (checked on the host before launch).
constexpr int64_t kRtMaxL = int64_t(1) << 53;       // L, so 511 L < 2^63
constexpr int64_t kRtMaxInvNum = int64_t(1) << 61;  // |exact inverse numerator|
constexpr int64_t kRtMaxQuantY = int64_t(1) << 24;  // |Y| with a quantiser

adct_status launch_codec_rt(int band, bool quant, bool float_in, Mode mode, const CodecArgs &a,
                            const RtMatArgs &m, int total_waves, hipStream_t s);

adct_status launch_dct(Mode mode, const DctArgs &a, int total_waves, hipStream_t s);

// Free the grow-only device buffers of the searches and of the coding-gain
// sweep on device `dev`; each returns the bytes it released.
int64_t release_search_cache(int dev);
int64_t release_gain_cache(int dev);

// Codec launch schedule: resident 4-wave workgroups per CU (0 = as many as
// occupancy allows, -1 = one tile per wave, no persistence).
int codec_wgs_per_cu();

adct_status launch_codec(int tid, int band, bool quant, Mode mode, const CodecArgs &a,
                         const QuantTables &q, int total_waves, hipStream_t s);

}  // namespace adct
