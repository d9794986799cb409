// Non-orthogonal low-complexity matrices (the signed DCT, BAS-2008b, any
// invertible integer T) on gfx950, and the unified coding gain against the
// inter-pixel correlation (Sec. 2, 4.2.3, 4.3, 6.1.1).
//
// Decoder: for T without orthogonal rows the transpose is no inverse, and the
// reconstruction is A = C_hat^-1 B' C_hat^-T.  With C_hat = S T (S diagonal) and
// zonal coding B' = S Y' S, this is T^-1 Y' T^-T = adj(T) Y' adj(T)^T / det(T)^2:
// with adj(T) and det(T) first divided by their common factor, so the signed
// DCT and BAS-2008b reconstruct over 8^2 instead of 2048^2 and 1024^2.  Where
// that denominator is a power of two and the numerators stay below 2^24 (both
// of those matrices) every step is exact in float32 and one conversion rounds
// and saturates; otherwise the kernel computes the numerator in float64 on
// integers (exact below 2^53, bounded on the host) and divides exactly.  Either way the pixels
// are bit-exact.  One lane owns one 8x8 block for the whole pipeline.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <vector>

#include "adct_internal.hpp"
#include "wave.hpp"

namespace adct {
namespace {

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

struct InvPlane {
    int64_t off;
    int32_t pitch, nbx, nblocks, wave_start;
    uint32_t nbx_m;        // b / nbx = umulhi(b, nbx_m) >> nbx_s (magic_u31)
    int32_t nbx_s;
};

struct InvArgs {
    const uint8_t *in;
    uint8_t *out;
    unsigned long long *sse;
    int64_t fs_in, fs_out;
    int32_t n_frames, n_planes, waves_per_frame, r;
    uint32_t wpf_m;        // gw / waves_per_frame by multiply-high (magic_u31)
    int32_t wpf_s;
    int32_t T[64];         // T[8k + m]
    double adj[64];        // adj(T)[8x + k] / g (g: the common factor of adj(T) and det(T))
    double den;            // (det(T) / g)^2
    double inv_den;
    int8_t T8[64];         // exact float32 form: T as bytes (four a scalar register)
    float adj_f[64];       //   the reduced adj(T)
    int32_t yoff[64];      //   128 (sum_m T[k][m]) (sum_m T[l][m]): Y minus Y of the pixels - 128
    float inv_den_f;       //   1 / den = 2^-e
    InvPlane pl[kMaxPlanes];
};

__device__ __forceinline__ unsigned wave_sum(unsigned v) { return wave_sum_u32(v); }

// round-half-to-even(n / den) clipped to [0, 255]; n and den integers held
// exactly in doubles
__device__ __forceinline__ int rne_div_exact(double n, double den, double inv_den) {
    const double c = fmin(fmax(n, 0.0), 255.0 * den);
    double q = floor(c * inv_den);
    double rem = c - q * den;
    if (rem < 0.0) { q -= 1.0; rem += den; }
    if (rem >= den) { q += 1.0; rem -= den; }
    const int qi = int(q);
    const double twice = rem + rem;
    return qi + ((twice > den || (twice == den && (qi & 1))) ? 1 : 0);
}

// BAND: only coefficients (k, l) with k + l <= BAND can be kept (r <= 10 needs
// BAND 3; 14 is the whole block); the products that only reach discarded
// coefficients or columns drop out at compile time.
template <int BAND>
__global__ __launch_bounds__(256) void k_inverse_codec(const InvArgs a) {
    constexpr int KB = BAND + 1 < 8 ? BAND + 1 : 8;     // columns (and rows) that can hold kept coefficients
    const int lane = threadIdx.x & 63;
    const int total = a.n_frames * a.waves_per_frame;
    unsigned long long acc = 0;
    int acc_fp = -1;
    // the wave index from the first lane: tile, frame and plane are then known
    // to be wave-uniform and stay on the scalar unit
    for (int gw = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)); gw < total;
         gw += int(gridDim.x) * 4) {
        const int f = gw / a.waves_per_frame;
        const int w = gw - f * a.waves_per_frame;
        int p = 0;
        while (p + 1 < a.n_planes && w >= a.pl[p + 1].wave_start) ++p;
        const InvPlane &P = a.pl[p];
        const int blk = (w - P.wave_start) * 64 + lane;
        const bool active = blk < P.nblocks;
        const int b = active ? blk : 0;
        const int by = b / P.nbx, bx = b - (b / P.nbx) * P.nbx;
        const int64_t off = P.off + int64_t(8 * by) * P.pitch + 8 * bx;
        const uint8_t *src = a.in + int64_t(f) * a.fs_in + off;
        uint32_t pix[8][2];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            const u32x2 v = *(const u32x2 *)(src + int64_t(x) * P.pitch);
            pix[x][0] = v.x;
            pix[x][1] = v.y;
        }
        // Y = T A T^T, then the zig-zag prefix
        int Z[8][KB];
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                int s = 0;
#pragma unroll
                for (int m = 0; m < 8; ++m) s += a.T[8 * l + m] * int((pix[x][m >> 2] >> (8 * (m & 3))) & 0xffu);
                Z[x][l] = s;
            }
        int Y[KB][KB];
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                int s = 0;
                if (k + l <= BAND) {
#pragma unroll
                    for (int x = 0; x < 8; ++x) s += a.T[8 * k + x] * Z[x][l];
                }
                Y[k][l] = (k + l <= BAND && zz_pos(k, l) < a.r) ? s : 0;
            }
        // numerator adj Y' adj^T row by row (integers, exact in float64); the
        // row loop stays rolled (one row's sums live at a time) and re-reads the
        // row's pixels for the error
        unsigned e = 0;
        uint8_t *dst = a.out ? a.out + int64_t(f) * a.fs_out + off : nullptr;
#pragma unroll 1
        for (int x = 0; x < 8; ++x) {
            const u32x2 px = *(const u32x2 *)(src + int64_t(x) * P.pitch);
            double U[KB];
#pragma unroll
            for (int l = 0; l < KB; ++l) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (k + l <= BAND) s = fma(a.adj[8 * x + k], double(Y[k][l]), s);
                U[l] = s;
            }
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int y = 0; y < 8; ++y) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < KB; ++l) s = fma(U[l], a.adj[8 * y + l], s);
                const int q = rne_div_exact(s, a.den, a.inv_den);
                const int d = q - int(((y < 4 ? px.x : px.y) >> (8 * (y & 3))) & 0xffu);
                e += unsigned(d * d);
                if (y < 4) lo |= uint32_t(q) << (8 * y); else hi |= uint32_t(q) << (8 * (y - 4));
            }
            if (active && dst) {
                u32x2 v;
                v.x = lo;
                v.y = hi;
                *(u32x2 *)(dst + int64_t(x) * P.pitch) = v;
            }
        }
        if (!active) e = 0;
        const int fp = f * a.n_planes + p;
        if (fp != acc_fp) {
            if (acc_fp >= 0 && acc && lane == 0) atomicAdd(a.sse + acc_fp, acc);
            acc = 0;
            acc_fp = fp;
        }
        acc += wave_sum(e);
    }
    if (acc_fp >= 0 && acc && lane == 0) atomicAdd(a.sse + acc_fp, acc);
}

// ------------------------------------------------------------------ exact float32 form
//
// For den = 2^e with every numerator below 2^24 in magnitude (the signed DCT
// and BAS-2008b after the common factor is divided out): Y / den, its products
// with adj and their sums are multiples of 2^-e below 2^24 2^-e, so float32
// holds every step exactly, and the pixel is one conversion that rounds half
// to even and saturates to [0, 255].

struct InvBlock {
    int f, p;
    bool active;
    int64_t off;           // byte offset of the block's top-left pixel inside a frame
};

// n / d for 0 <= n < 2^31 from the magic pair of d
__device__ __forceinline__ int udiv_magic(int n, uint32_t m, int s) {
    return s < 0 ? n : int(__umulhi(uint32_t(n), m) >> s);
}

// The frame, plane and first block are wave-uniform and stay on the scalar
// unit (multiply-high divisions by host-computed magic numbers); a lane's
// block row is one more multiply-high, its offset inside the plane 32 bits
// (the host bounds H and the pitch below 2^24 and a plane below 2^31 bytes).
__device__ __forceinline__ InvBlock inv_block_of(const InvArgs &a, int gw, int lane) {
    InvBlock B;
    B.f = __builtin_amdgcn_readfirstlane(udiv_magic(gw, a.wpf_m, a.wpf_s));
    const int w = __builtin_amdgcn_readfirstlane(gw - B.f * a.waves_per_frame);
    int p = 0;
    while (p + 1 < a.n_planes && w >= a.pl[p + 1].wave_start) ++p;
    B.p = __builtin_amdgcn_readfirstlane(p);
    const InvPlane &P = a.pl[B.p];
    const int blk = (w - P.wave_start) * 64 + lane;
    B.active = blk < P.nblocks;
    const int b = B.active ? blk : 0;       // idle lanes read block 0 of the plane
    const int by = udiv_magic(b, P.nbx_m, P.nbx_s), bx = b - by * P.nbx;
    B.off = P.off + (__umul24(uint32_t(8 * by), uint32_t(P.pitch)) + uint32_t(8 * bx));
    return B;
}

__device__ __forceinline__ void inv_load(const InvArgs &a, const InvBlock &B, uint32_t (&pix)[8][2]) {
    const int pitch = a.pl[B.p].pitch;
    const uint8_t *src = a.in + int64_t(B.f) * a.fs_in + B.off;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const u32x2 v = __builtin_nontemporal_load((const u32x2 *)(src + int64_t(x) * pitch));
        pix[x][0] = v.x;
        pix[x][1] = v.y;
    }
}

template <int BAND>
__device__ __forceinline__ void inv_int_block(const InvArgs &a, const InvBlock &B, const uint32_t (&pix)[8][2],
                                              unsigned long long &acc, int &acc_fp) {
    constexpr int KB = BAND + 1 < 8 ? BAND + 1 : 8;
    const int lane = threadIdx.x & 63;
    // Y = T A T^T, then the zig-zag prefix.  The row pass takes the pixels
    // minus 128 as signed bytes, four products per signed dot instruction
    // against a packed row of T; the constant the offset adds to Y is yoff.
    const int32_t *tpk = reinterpret_cast<const int32_t *>(a.T8);
    int Z[8][KB];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const int p0 = int(pix[x][0] ^ 0x80808080u), p1 = int(pix[x][1] ^ 0x80808080u);
#pragma unroll
        for (int l = 0; l < KB; ++l)
            Z[x][l] = __builtin_amdgcn_sdot4(tpk[2 * l + 1], p1, __builtin_amdgcn_sdot4(tpk[2 * l], p0, 0, false),
                                             false);
    }
    int Y[KB][KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int l = 0; l < KB; ++l) {
            int s = 0;
            if (k + l <= BAND) {
                s = a.yoff[8 * k + l];
#pragma unroll
                for (int x = 0; x < 8; ++x) s += __mul24(int(a.T8[8 * k + x]), Z[x][l]);
            }
            Y[k][l] = (k + l <= BAND && zz_pos(k, l) < a.r) ? s : 0;
        }
    // (adj Y' adj^T) / den row by row in exact float32
    float Yf[KB][KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int l = 0; l < KB; ++l) Yf[k][l] = (k + l <= BAND) ? float(Y[k][l]) * a.inv_den_f : 0.f;
    uint8_t *dst = a.out ? a.out + int64_t(B.f) * a.fs_out + B.off : nullptr;
    const int pitch = a.pl[B.p].pitch;
    uint32_t sq = 0, cross = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        float U[KB];
#pragma unroll
        for (int l = 0; l < KB; ++l) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (k + l <= BAND) s = fmaf(a.adj_f[8 * x + k], Yf[k][l], s);
            U[l] = s;
        }
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            float s = 0.f;
#pragma unroll
            for (int l = 0; l < KB; ++l) s = fmaf(U[l], a.adj_f[8 * y + l], s);
            w[y >> 2] = __builtin_amdgcn_cvt_pk_u8_f32(s, uint32_t(y & 3), w[y >> 2]);
        }
        u32x2 v;
        v.x = w[0];
        v.y = w[1];
        sq = __builtin_amdgcn_udot4(v.x, v.x, sq, false);
        sq = __builtin_amdgcn_udot4(v.y, v.y, sq, false);
        sq = __builtin_amdgcn_udot4(pix[x][0], pix[x][0], sq, false);
        sq = __builtin_amdgcn_udot4(pix[x][1], pix[x][1], sq, false);
        cross = __builtin_amdgcn_udot4(v.x, pix[x][0], cross, false);
        cross = __builtin_amdgcn_udot4(v.y, pix[x][1], cross, false);
        if (B.active && dst) __builtin_nontemporal_store(v, (u32x2 *)(dst + int64_t(x) * pitch));
    }
    // sum (q - a)^2 = sum q^2 + sum a^2 - 2 sum q a (exact modulo 2^32, below it)
    const unsigned e = B.active ? sq - 2u * cross : 0u;
    const int fp = B.f * a.n_planes + B.p;
    if (fp != acc_fp) {
        if (acc_fp >= 0 && acc && lane == 0) atomicAdd(a.sse + acc_fp, acc);
        acc = 0;
        acc_fp = fp;
    }
    acc += wave_sum(e);
}

// Persistent grid; each wave loads its next 64 blocks before it transforms
// the current ones (on every pass: the last pass re-reads its own blocks).
template <int BAND>
__global__ __launch_bounds__(256) void k_inverse_int(const InvArgs a) {
    const int lane = threadIdx.x & 63;
    const int total = a.n_frames * a.waves_per_frame;
    const int stride = int(gridDim.x) * 4;
    int gw = int(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    if (gw >= total) return;
    unsigned long long acc = 0;
    int acc_fp = -1;
    uint32_t pa[8][2], pb[8][2];
    InvBlock ba = inv_block_of(a, gw, lane), bb = ba;
    inv_load(a, ba, pa);
    while (true) {
        int nxt = gw + stride;
        bool more = nxt < total;                  // wave-uniform
        bb = inv_block_of(a, more ? nxt : gw, lane);
        inv_load(a, bb, pb);
        inv_int_block<BAND>(a, ba, pa, acc, acc_fp);
        if (!more) break;
        gw = nxt;
        nxt = gw + stride;
        more = nxt < total;
        ba = inv_block_of(a, more ? nxt : gw, lane);
        inv_load(a, ba, pa);
        inv_int_block<BAND>(a, bb, pb, acc, acc_fp);
        if (!more) break;
        gw = nxt;
    }
    if (acc_fp >= 0 && acc && lane == 0) atomicAdd(a.sse + acc_fp, acc);
}

__global__ void k_inv_zero(unsigned long long *p, int n) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0ull;
}

// ------------------------------------------------------------------ coding gain

// C_g*(C_hat, rho) = 10 sum_i -log10(A_i B_i) / 8 with A_i = sum_jk c_ij c_ik
// rho^|j - k| and B_i the squared norm of row i of C_hat^-1 (Sec. 4.2.3).  One
// thread per (matrix, rho); the inverse by Gauss-Jordan with partial pivoting.
__global__ void k_coding_gain(const double *c_hat, int n_t, const double *rho, int n_rho, double *out) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_t * n_rho) return;
    const int t = i / n_rho, j = i - t * n_rho;
    const double *c = c_hat + 64 * t;
    double m[8][16];
    for (int r = 0; r < 8; ++r)
        for (int q = 0; q < 16; ++q) m[r][q] = q < 8 ? c[8 * r + q] : (q - 8 == r ? 1.0 : 0.0);
    for (int col = 0; col < 8; ++col) {
        int piv = col;
        for (int r = col + 1; r < 8; ++r)
            if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
        if (piv != col)
            for (int q = 0; q < 16; ++q) {
                const double tmp = m[col][q];
                m[col][q] = m[piv][q];
                m[piv][q] = tmp;
            }
        const double inv = 1.0 / m[col][col];
        for (int q = 0; q < 16; ++q) m[col][q] *= inv;
        for (int r = 0; r < 8; ++r) {
            if (r == col) continue;
            const double fct = m[r][col];
            for (int q = 0; q < 16; ++q) m[r][q] -= fct * m[col][q];
        }
    }
    double pw[8];
    pw[0] = 1.0;
    for (int d = 1; d < 8; ++d) pw[d] = pw[d - 1] * rho[j];
    double total = 0.0;
    for (int r = 0; r < 8; ++r) {
        double A = 0.0, B = 0.0;
        for (int x = 0; x < 8; ++x)
            for (int y = 0; y < 8; ++y) A += c[8 * r + x] * c[8 * r + y] * pw[x > y ? x - y : y - x];
        for (int q = 0; q < 8; ++q) B += m[r][8 + q] * m[r][8 + q];
        total += -log10(A * B) / 8.0;
    }
    out[i] = 10.0 * total;
}

// exact determinant of an n x n integer matrix (n <= 8) by fraction-free
// (Bareiss) elimination: every division is exact
__int128 bareiss_det(__int128 (*m)[8], int n) {
    __int128 prev = 1;
    int sign = 1;
    for (int k = 0; k < n - 1; ++k) {
        if (m[k][k] == 0) {
            int r = k + 1;
            while (r < n && m[r][k] == 0) ++r;
            if (r == n) return 0;
            for (int q = 0; q < n; ++q) std::swap(m[k][q], m[r][q]);
            sign = -sign;
        }
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) m[i][j] = (m[i][j] * m[k][k] - m[i][k] * m[k][j]) / prev;
        prev = m[k][k];
    }
    return sign * m[n - 1][n - 1];
}

// adj(T) (the transposed cofactor matrix, adj(T) T = det(T) I) and det(T):
// 0 on success, 1 when T is singular, 2 when an entry reaches 2^53
int adjugate_det(const int8_t *T, int64_t adj[64], int64_t *det) {
    const __int128 lim = __int128(1) << 53;
    __int128 m[8][8];
    for (int r = 0; r < 8; ++r)
        for (int q = 0; q < 8; ++q) m[r][q] = T[8 * r + q];
    const __int128 d = bareiss_det(m, 8);
    if (d == 0) return 1;
    if (d >= lim || d <= -lim) return 2;
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            // cofactor C_ji: delete row j and column i
            __int128 mm[8][8];
            for (int r = 0, rr = 0; r < 8; ++r) {
                if (r == j) continue;
                for (int q = 0, qq = 0; q < 8; ++q) {
                    if (q == i) continue;
                    mm[rr][qq++] = T[8 * r + q];
                }
                ++rr;
            }
            const __int128 c = bareiss_det(mm, 7);
            if (c >= lim || c <= -lim) return 2;
            adj[8 * i + j] = int64_t(((i + j) & 1) ? -c : c);
        }
    *det = int64_t(d);
    return 0;
}

// The adjugate takes 64 fraction-free 7 x 7 eliminations in 128-bit integers,
// tens of microseconds of host time per call: each thread keeps the last few
// results keyed by the matrix bytes (callers repeat one matrix over images).
struct AdjEntry {
    bool valid = false;
    int8_t T[64];
    int status;
    int64_t adj[64], det;
};
constexpr int kAdjSlots = 4;
thread_local AdjEntry g_adj[kAdjSlots];
thread_local int g_adj_next = 0;

int adjugate_det_cached(const int8_t *T, int64_t adj[64], int64_t *det) {
    for (const AdjEntry &e : g_adj)
        if (e.valid && memcmp(e.T, T, 64) == 0) {
            memcpy(adj, e.adj, sizeof(e.adj));
            *det = e.det;
            return e.status;
        }
    AdjEntry &e = g_adj[g_adj_next];
    g_adj_next = (g_adj_next + 1) % kAdjSlots;
    e.status = adjugate_det(T, e.adj, &e.det);
    memcpy(e.T, T, 64);
    e.valid = true;
    memcpy(adj, e.adj, sizeof(e.adj));
    *det = e.det;
    return e.status;
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" adct_status adct_evaluate_inverse(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                             const adct_plane *planes, int n_planes, const int8_t *T, int r,
                                             uint8_t *recon, int64_t frame_stride_out, uint64_t *sse,
                                             adct_stream_t stream) {
    if (!frames || !planes || !T || !sse) return fail(ADCT_EINVAL, "frames, planes, T and sse are required");
    if (r < 1 || r > 64) return fail(ADCT_ERANGE, "r must be in [1, 64]");
    if (n_frames < 1) return fail(ADCT_ERANGE, "n_frames must be >= 1");
    if (n_planes < 1 || n_planes > kMaxPlanes) return fail(ADCT_ERANGE, "n_planes must be in [1, 4]");
    if (n_frames > 1 && (frame_stride <= 0 || (recon && frame_stride_out <= 0)))
        return fail(ADCT_EDIM, "frame strides must be positive for several frames");
    if (reinterpret_cast<uintptr_t>(sse) & 7) return fail(ADCT_EDIM, "sse must be 8-byte aligned");
    InvArgs a;
    memset(&a, 0, sizeof(a));
    int64_t adj[64], det = 0;
    const int ad = adjugate_det_cached(T, adj, &det);
    if (ad == 1) return fail(ADCT_EINVAL, "T is singular");
    if (ad == 2) return fail(ADCT_EOVERFLOW, "T is too large for exact float64 numerators");
    // T^-1 = adj / det: divide out the common factor of all entries and det
    int64_t g = det < 0 ? -det : det;
    for (int i = 0; i < 64; ++i) g = std::gcd(g, adj[i] < 0 ? -adj[i] : adj[i]);
    for (int i = 0; i < 64; ++i) adj[i] /= g;
    det /= g;
    // numerator bound: |adj Y' adj^T| <= (sum |adj|)^2 max|Y| per entry
    int64_t rowsum = 0, tsum = 0;
    for (int k = 0; k < 8; ++k) {
        int64_t s = 0, u = 0;
        for (int m = 0; m < 8; ++m) {
            s += std::abs(int64_t(T[8 * k + m]));
            u += std::abs(adj[8 * k + m]);
        }
        tsum = std::max(tsum, s);
        rowsum = std::max(rowsum, u);
    }
    const double ymax = 255.0 * double(tsum) * double(tsum);
    if (double(rowsum) * double(rowsum) * ymax >= 9.0e15 || double(det) * double(det) >= 9.0e15 ||
        ymax * 8 >= 2.0e9)
        return fail(ADCT_EOVERFLOW, "T is too large for exact float64 numerators");
    for (int i = 0; i < 64; ++i) {
        a.T[i] = T[i];
        a.adj[i] = double(adj[i]);
    }
    a.den = double(det) * double(det);
    a.inv_den = 1.0 / a.den;
    // the exact float32 form: den a power of two, every numerator (Y, the row
    // sums U, the pixel sums) below 2^24; Y in int32 products of 24-bit operands
    const int64_t den = det * det;
    const int64_t ymax_i = 255 * tsum * tsum, umax = rowsum * ymax_i, smax = rowsum * umax;
    const bool int_form = (den & (den - 1)) == 0 && smax < (int64_t(1) << 24) && umax < (int64_t(1) << 24) &&
                          ymax_i < (int64_t(1) << 23);
    if (int_form) {
        int rs[8] = {};
        for (int i = 0; i < 64; ++i) {
            a.T8[i] = T[i];
            a.adj_f[i] = float(adj[i]);
            rs[i / 8] += T[i];
        }
        for (int i = 0; i < 64; ++i) a.yoff[i] = 128 * rs[i / 8] * rs[i % 8];
        a.inv_den_f = float(1.0 / double(den));
    }
    a.in = frames;
    a.out = recon;
    a.sse = reinterpret_cast<unsigned long long *>(sse);
    a.fs_in = frame_stride;
    a.fs_out = frame_stride_out;
    a.n_frames = n_frames;
    a.n_planes = n_planes;
    a.r = r;
    int64_t waves = 0;
    for (int p = 0; p < n_planes; ++p) {
        const adct_plane &q = planes[p];
        if (q.H < 8 || q.W < 8 || (q.H & 7) || (q.W & 7) || q.pitch < q.W || q.offset < 0)
            return fail(ADCT_EDIM, "each plane needs H, W positive multiples of 8, pitch >= W, offset >= 0");
        if (q.H >= (1 << 24) || q.pitch >= (1 << 24) || int64_t(q.H) * q.pitch >= (int64_t(1) << 31))
            return fail(ADCT_ERANGE, "planes are limited to H, pitch < 2^24 and H * pitch < 2^31");
        InvPlane &d = a.pl[p];
        d.off = q.offset;
        d.pitch = q.pitch;
        d.nbx = q.W / 8;
        magic_u31(uint32_t(d.nbx), &d.nbx_m, &d.nbx_s);
        d.nblocks = (q.H / 8) * (q.W / 8);
        d.wave_start = int32_t(waves);
        waves += (d.nblocks + 63) / 64;
        if (waves > (int64_t(1) << 30)) return fail(ADCT_ERANGE, "planes too large");
    }
    if (waves * n_frames > (int64_t(1) << 31) - 1) return fail(ADCT_ERANGE, "too many blocks in one call");
    a.waves_per_frame = int32_t(waves);
    magic_u31(uint32_t(waves), &a.wpf_m, &a.wpf_s);
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int nz = n_frames * n_planes;
    hipLaunchKernelGGL(k_inv_zero, dim3((nz + 255) / 256), dim3(256), 0, hs, a.sse, nz);
    ADCT_HIP(hipGetLastError());
    int dev = 0, cus = 0, per_cu = 0;
    ADCT_HIP(hipGetDevice(&dev));
    ADCT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // r <= 10 keeps only coefficients with k + l <= 3
    auto kern = int_form ? (r <= 10 ? k_inverse_int<3> : k_inverse_int<14>)
                         : (r <= 10 ? k_inverse_codec<3> : k_inverse_codec<14>);
    ADCT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
    const int64_t want = (waves * n_frames + 3) / 4;
    const int grid = int(std::min<int64_t>(want, int64_t(std::max(per_cu, 1)) * cus));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, hs, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

// One grow-only staging buffer per device for adct_coding_gain_sweep (the
// call synchronises its stream before it returns, so the next call on the
// device may reuse it); the lock serialises calls on one device.
struct GainCache {
    std::mutex lock;
    void *p = nullptr;
    size_t bytes = 0;
};
GainCache g_gain[64];

int64_t adct::release_gain_cache(int dev) {
    if (dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> hold(g_gain[dev].lock);
    const int64_t n = int64_t(g_gain[dev].bytes);
    if (g_gain[dev].p) (void)hipFree(g_gain[dev].p);
    g_gain[dev].p = nullptr;
    g_gain[dev].bytes = 0;
    return n;
}

extern "C" adct_status adct_coding_gain_sweep(const double *c_hat, int n_t, const double *rho, int n_rho,
                                              double *cg_out, adct_stream_t stream) {
    if (!c_hat || !rho || !cg_out) return fail(ADCT_EINVAL, "c_hat, rho and cg_out are required");
    if (n_t < 1 || n_rho < 1 || int64_t(n_t) * n_rho > (int64_t(1) << 26))
        return fail(ADCT_ERANGE, "n_t and n_rho must be >= 1, n_t * n_rho <= 2^26");
    for (int j = 0; j < n_rho; ++j)
        if (!(rho[j] >= 0.0 && rho[j] < 1.0)) return fail(ADCT_ERANGE, "rho must be in [0, 1)");
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const size_t nc = size_t(n_t) * 64, no = size_t(n_t) * n_rho;
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(ADCT_EDEVICE, "device index beyond the library's table");
    GainCache &gc = g_gain[dev];
    std::lock_guard<std::mutex> hold(gc.lock);
    const size_t need = (nc + size_t(n_rho) + no) * sizeof(double);
    if (gc.bytes < need) {
        if (gc.p) (void)hipFree(gc.p);
        gc.p = nullptr;
        gc.bytes = 0;
        ADCT_HIP(hipMalloc(&gc.p, need));
        gc.bytes = need;
    }
    double *dc = static_cast<double *>(gc.p), *dr = dc + nc, *dout = dr + n_rho;
    adct_status st = ADCT_OK;
    hipError_t e = hipMemcpyAsync(dc, c_hat, nc * sizeof(double), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(dr, rho, size_t(n_rho) * sizeof(double), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_coding_gain, dim3(unsigned((no + 255) / 256)), dim3(256), 0, hs, dc, n_t, dr, n_rho,
                           dout);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(cg_out, dout, no * sizeof(double), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) st = hip_fail(e, "coding gain sweep");
    return st;
}

// ---------------------------------------------------------------- no-allocation form
//
// The same sweep for callers that cannot allocate device memory: the staged
// matrices, correlations and results live in one file-scope device array of a
// fixed size, held by each GPU the library runs on until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: every
// host use goes through the device address that hipGetSymbolAddress returns,
// taken once per device with that device current.

namespace {

constexpr int64_t kCgScratchDoubles = int64_t(1) << 18;   // 2 MiB per device
static __device__ __align__(256) double scratch[kCgScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

adct_status scratch_of_current_device(double **out) {
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ADCT_EDEVICE, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        ADCT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ADCT_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return ADCT_OK;
}

}  // namespace

extern "C" adct_status adct_coding_gain_sweep_noalloc(const double *c_hat, int n_t, const double *rho,
                                                      int n_rho, double *cg_out, adct_stream_t stream) {
    if (!c_hat || !rho || !cg_out) return fail(ADCT_EINVAL, "c_hat, rho and cg_out are required");
    if (n_t < 1 || n_rho < 1) return fail(ADCT_ERANGE, "n_t and n_rho must be >= 1");
    const int64_t nc = int64_t(n_t) * 64, no = int64_t(n_t) * n_rho;
    if (nc + n_rho + no > kCgScratchDoubles)
        return fail(ADCT_ERANGE, "64 n_t + n_rho + n_t n_rho must not exceed 262,144 doubles "
                                 "(the fixed scratch of the no-allocation sweep)");
    for (int j = 0; j < n_rho; ++j)
        if (!(rho[j] >= 0.0 && rho[j] < 1.0)) return fail(ADCT_ERANGE, "rho must be in [0, 1)");
    double *base = nullptr;
    adct_status st = scratch_of_current_device(&base);
    if (st) return st;
    double *dc = base, *dr = base + nc, *dout = base + nc + n_rho;   // every entry written before use
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    ADCT_HIP(hipMemcpyAsync(dc, c_hat, size_t(nc) * sizeof(double), hipMemcpyHostToDevice, hs));
    ADCT_HIP(hipMemcpyAsync(dr, rho, size_t(n_rho) * sizeof(double), hipMemcpyHostToDevice, hs));
    hipLaunchKernelGGL(k_coding_gain, dim3(unsigned((no + 255) / 256)), dim3(256), 0, hs, dc, n_t, dr, n_rho,
                       dout);
    ADCT_HIP(hipGetLastError());
    ADCT_HIP(hipMemcpyAsync(cg_out, dout, size_t(no) * sizeof(double), hipMemcpyDeviceToHost, hs));
    ADCT_HIP(hipStreamSynchronize(hs));
    return ADCT_OK;
}
