// Exact signs in Q(sqrt p, sqrt q) for the rounding of dequantised
// reconstructions near a half.  Host and device functions: the same source is
// what the kernels run and what the CPU tests check against exact arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adct {

typedef __int128 i128;
typedef unsigned __int128 u128;

struct U256 {
    uint64_t w[4];
};

// a b for a, b < 2^128
__host__ __device__ inline U256 mul_u128(u128 a, u128 b) {
    const uint64_t a0 = uint64_t(a), a1 = uint64_t(a >> 64), b0 = uint64_t(b), b1 = uint64_t(b >> 64);
    const u128 p00 = u128(a0) * b0, p01 = u128(a0) * b1, p10 = u128(a1) * b0, p11 = u128(a1) * b1;
    const u128 mid = (p00 >> 64) + uint64_t(p01) + uint64_t(p10);
    const u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + uint64_t(p11);
    U256 r;
    r.w[0] = uint64_t(p00);
    r.w[1] = uint64_t(mid);
    r.w[2] = uint64_t(hi);
    r.w[3] = uint64_t(hi >> 64) + uint64_t(p11 >> 64);
    return r;
}

// a s for a small s (the product stays below 2^256)
__host__ __device__ inline U256 mul_small(const U256 &a, uint32_t s) {
    U256 r;
    u128 c = 0;
    for (int i = 0; i < 4; ++i) {
        c += u128(a.w[i]) * s;
        r.w[i] = uint64_t(c);
        c >>= 64;
    }
    return r;
}

__host__ __device__ inline int cmp256(const U256 &a, const U256 &b) {
    for (int i = 3; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] > b.w[i] ? 1 : -1;
    return 0;
}

__host__ __device__ inline int sgn128(i128 v) { return (v > 0) - (v < 0); }
__host__ __device__ inline u128 abs128(i128 v) { return v < 0 ? u128(-v) : u128(v); }

// sign of a + b sqrt(p), p > 1 squarefree, |a|, |b| < 2^127: with opposite
// signs the larger of a^2 and p b^2 decides
__host__ __device__ inline int sgn_surd(i128 a, i128 b, uint32_t p) {
    const int sa = sgn128(a), sb = sgn128(b);
    if (sb == 0) return sa;
    if (sa == 0 || sa == sb) return sa == 0 ? sb : sa;
    const int c = cmp256(mul_u128(abs128(a), abs128(a)), mul_small(mul_u128(abs128(b), abs128(b)), p));
    return c > 0 ? sa : c < 0 ? sb : 0;
}

// sign of X + Y sqrt(q) with X = a + b sqrt(p), Y = c + d sqrt(p) (q = 1: no
// second generator, c = d = 0): with opposite signs the sign of
// X^2 - q Y^2 = E + F sqrt(p) decides.  Components below 2^52 and p q <= 1024
// keep E and F below 2^127 and their squares below 2^256.
__host__ __device__ inline int sgn_field(i128 a, i128 b, i128 c, i128 d, uint32_t p, uint32_t q) {
    const int sx = sgn_surd(a, b, p);
    if (q <= 1) return sx;
    const int sy = sgn_surd(c, d, p);
    if (sx == 0 || sy == 0 || sx == sy) return sx == 0 ? sy : sx;
    const i128 E = a * a + i128(p) * b * b - i128(q) * (c * c + i128(p) * d * d);
    const i128 F = 2 * (a * b - i128(q) * c * d);
    const int s = sgn_surd(E, F, p);
    return s > 0 ? sx : s < 0 ? sy : 0;
}

}  // namespace adct
