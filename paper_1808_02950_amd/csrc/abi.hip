// C ABI entry points: argument validation, constant set-up and dispatch.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "adct_internal.hpp"

namespace adct {

static thread_local std::string g_err;
static int g_codec_wgs_per_cu = 0;

int codec_wgs_per_cu() { return g_codec_wgs_per_cu; }

void set_error(const std::string &msg) { g_err = msg; }

adct_status fail(adct_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

adct_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return ADCT_EDEVICE;
}

namespace {

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Small fill kernel instead of hipMemsetAsync so the call stays graph-safe.
adct_status zero_u64(uint64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return ADCT_OK;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u64, dim3(unsigned(blocks)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(p), n, 0ull);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

bool is_builtin_int(int t) { return t >= ADCT_T1 && t <= ADCT_T4; }

void matrix_of(int t, adct_matrix *m) {
    const Mat8 &src = builtin(t);
    for (int k = 0; k < 8; ++k) {
        int32_t s = 0;
        for (int c = 0; c < 8; ++c) {
            m->T[8 * k + c] = src.m[k][c];
            s += int32_t(src.m[k][c]) * src.m[k][c];
        }
        m->n[k] = s;
    }
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Exact bound of |Y_kl| over 8-bit blocks, max over (k, l).
int64_t fwd_bound(const adct_matrix &m) {
    int64_t best = 0;
    for (int k = 0; k < 8; ++k)
        for (int l = 0; l < 8; ++l) {
            int64_t pos = 0, neg = 0;
            for (int u = 0; u < 8; ++u)
                for (int v = 0; v < 8; ++v) {
                    const int64_t c = int64_t(m.T[8 * k + u]) * m.T[8 * l + v];
                    if (c > 0) pos += c; else neg -= c;
                }
            best = std::max(best, 255 * std::max(pos, neg));
        }
    return best;
}

int64_t lcm64(int64_t a, int64_t b) {
    int64_t x = a, y = b;
    while (y) { const int64_t t = x % y; x = y; y = t; }
    return a / x * b;
}

// Exact bound of the inverse numerator T^T (Y' o c c^T) T over 8-bit blocks for
// the zig-zag prefix of length r, c_k = lcm(n) / n_k; saturates at INT64_MAX
// (a caller's matrix can have a large lcm).
int64_t inv_bound(const adct_matrix &m, int r) {
    __int128 l1 = 1;
    for (int k = 0; k < 8; ++k) {
        __int128 x = l1, y = m.n[k];
        while (y) { const __int128 t = x % y; x = y; y = t; }
        l1 = l1 / x * m.n[k];
        if (l1 > (__int128(1) << 62)) return INT64_MAX;
    }
    __int128 c[8];
    for (int k = 0; k < 8; ++k) c[k] = l1 / m.n[k];
    const __int128 cap = __int128(INT64_MAX);
    __int128 best = 0;
    for (int x = 0; x < 8; ++x)
        for (int y = 0; y < 8; ++y) {
            __int128 kern[64] = {0};
            for (int z = 0; z < r; ++z) {
                const int k = kZZ[z] >> 3, l = kZZ[z] & 7;
                const __int128 w = c[k] * c[l] * m.T[8 * k + x] * m.T[8 * l + y];
                if (!w) continue;
                if (w > cap || -w > cap) return INT64_MAX;
                for (int u = 0; u < 8; ++u)
                    for (int v = 0; v < 8; ++v) kern[8 * u + v] += w * m.T[8 * k + u] * m.T[8 * l + v];
            }
            __int128 pos = 0, neg = 0;
            for (int i = 0; i < 64; ++i) {
                if (kern[i] > 0) pos += kern[i]; else neg -= kern[i];
            }
            best = std::max(best, 255 * std::max(pos, neg));
            if (best > cap) return INT64_MAX;
        }
    return int64_t(best);
}

// A caller's matrix: n must be diag(T T^T), every row non-zero, rows orthogonal.
adct_status check_custom(const adct_matrix *c) {
    if (!c) return fail(ADCT_EINVAL, "ADCT_CUSTOM needs a matrix in `custom`");
    for (int k = 0; k < 8; ++k) {
        for (int l = 0; l < 8; ++l) {
            int64_t d = 0;
            for (int j = 0; j < 8; ++j) d += int64_t(c->T[8 * k + j]) * c->T[8 * l + j];
            if (k == l && (d == 0 || d != c->n[k]))
                return fail(ADCT_EINVAL, "custom matrix: n[k] must equal (T T^T)_kk > 0");
            if (k != l && d != 0)
                return fail(ADCT_EINVAL, "custom matrix: rows are not orthogonal (T T^T not diagonal); "
                                         "the transpose decoder of Sec. 6.1.1 needs orthogonal rows");
        }
    }
    return ADCT_OK;
}

// Run-time kernel constants of matrix m (all entries wave-uniform).
adct_status build_rt(const adct_matrix &m, RtMatArgs *rt) {
    int64_t l1 = 1;
    for (int k = 0; k < 8; ++k) {
        l1 = lcm64(l1, m.n[k]);
        if (l1 > (int64_t(1) << 26)) return fail(ADCT_EOVERFLOW, "lcm of the row norms exceeds 2^26");
    }
    memset(rt, 0, sizeof(*rt));
    rt->L = l1 * l1;
    if (rt->L >= kRtMaxL) return fail(ADCT_EOVERFLOW, "exact inverse denominator exceeds 2^53");
    rt->inv_2L = 1.0 / double(2 * rt->L);
    for (int k = 0; k < 8; ++k)
        for (int l = 0; l < 8; ++l) {
            const int i = 8 * k + l;
            rt->t[i] = m.T[i];
            const int64_t v = int64_t(m.n[k]) * m.n[l];
            const int64_t mu = int64_t(llround(sqrt(double(v))));
            rt->mu[i] = (mu * mu == v) ? int32_t(mu) : 0;
            rt->inv_2mu[i] = rt->mu[i] ? float(0.5 / double(rt->mu[i])) : 0.f;
            rt->ckl[i] = (l1 / m.n[k]) * (l1 / m.n[l]);
            rt->skl[i] = inv_sqrt_newton(v);
        }
    return ADCT_OK;
}

// The run-time exact inverse sums int64 terms T[k][x] c_k c_l C_kl into U[x][l],
// then T[l][y] U[x][l] into the numerator; with |C| <= cmax (the forward bound,
// or any int16 a decoder is handed) every partial sum must stay below 2^61,
// and the denominator L below 2^53.
bool rt_words_fit(const adct_matrix &m, int64_t cmax) {
    __int128 l1 = 1;
    for (int k = 0; k < 8; ++k) {
        __int128 x = l1, y = m.n[k];
        while (y) { const __int128 t = x % y; x = y; y = t; }
        l1 = l1 / x * m.n[k];
        if (l1 > (__int128(1) << 26)) return false;
    }
    if (l1 * l1 >= kRtMaxL) return false;
    __int128 umax = 0;
    for (int x = 0; x < 8; ++x)
        for (int l = 0; l < 8; ++l) {
            __int128 u = 0;
            for (int k = 0; k < 8; ++k)
                u += __int128(m.T[8 * k + x] < 0 ? -m.T[8 * k + x] : m.T[8 * k + x]) *
                     (l1 / m.n[k]) * (l1 / m.n[l]) * cmax;
            umax = std::max(umax, u);
        }
    __int128 nmax = 0;
    for (int y = 0; y < 8; ++y) {
        __int128 v = 0;
        for (int l = 0; l < 8; ++l) v += __int128(m.T[8 * l + y] < 0 ? -m.T[8 * l + y] : m.T[8 * l + y]) * umax;
        nmax = std::max(nmax, v);
    }
    return nmax < kRtMaxInvNum;
}

// Prime factorisation of 0 < v < 2^31 by trial division.
struct Fact {
    int n = 0;
    int64_t p[16];
    int e[16];
};
Fact factor(int64_t v) {
    Fact f;
    for (int64_t d = 2; d * d <= v; ++d) {
        if (v % d) continue;
        f.p[f.n] = d;
        f.e[f.n] = 0;
        while (v % d == 0) {
            v /= d;
            ++f.e[f.n];
        }
        ++f.n;
    }
    if (v > 1) {
        f.p[f.n] = v;
        f.e[f.n] = 1;
        ++f.n;
    }
    return f;
}

// squarefree part of a b and the mu with a b = mu^2 r
void split_square(const Fact &fa, const Fact &fb, int64_t *mu, int64_t *r) {
    int64_t m = 1, q = 1;
    int64_t ps[32];
    int es[32], n = 0;
    for (int i = 0; i < fa.n; ++i) { ps[n] = fa.p[i]; es[n++] = fa.e[i]; }
    for (int i = 0; i < fb.n; ++i) {
        int j = 0;
        while (j < n && ps[j] != fb.p[i]) ++j;
        if (j == n) { ps[n] = fb.p[i]; es[n++] = fb.e[i]; }
        else es[j] += fb.e[i];
    }
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < es[i] / 2; ++k) m *= ps[i];
        if (es[i] & 1) q *= ps[i];
    }
    *mu = m;
    *r = q;
}

int64_t squarefree(int64_t v) {
    int64_t mu, r;
    split_square(factor(v), Fact{}, &mu, &r);
    return r;
}

// Tables of the exact near-half decision for matrix m, zig-zag band `band`
// (coefficients k + l <= band) and a quantiser step: the squarefree parts of
// n_k n_l, two generators, the common denominator and weights, and the word
// bounds for any int16 levels a decoder may be handed.
adct_status build_settle(const adct_matrix &m, int band, int step, RtSettle *st) {
    memset(st, 0, sizeof(*st));
    Fact fn[8];
    for (int k = 0; k < 8; ++k) fn[k] = factor(m.n[k]);
    int64_t mu[64], rr[64];
    int64_t R[64];
    int nr = 0;
    for (int k = 0; k < 8; ++k)
        for (int l = 0; l < 8; ++l) {
            const int i = 8 * k + l;
            split_square(fn[k], fn[l], &mu[i], &rr[i]);
            if (k + l > band || rr[i] == 1) continue;
            int j = 0;
            while (j < nr && R[j] != rr[i]) ++j;
            if (j == nr) R[nr++] = rr[i];
        }
    int64_t p = 1, q = 1, r3 = 1;
    if (nr == 1) {
        p = R[0];
    } else if (nr > 1) {
        bool found = false;
        for (int i = 0; i < nr && !found; ++i)
            for (int j = i + 1; j < nr && !found; ++j) {
                const int64_t c = squarefree(R[i] * R[j]);
                bool all = true;
                for (int t = 0; t < nr; ++t) all &= R[t] == R[i] || R[t] == R[j] || R[t] == c;
                if (all) {
                    p = R[i];
                    q = R[j];
                    r3 = c;
                    found = true;
                }
            }
        if (!found)
            return fail(ADCT_ENOTSUP, "quant_step admits exact half ties and the row norms bring in more than "
                                      "two independent square roots: no exact decision of those halves");
    }
    if (p * q > kSettleMaxPQ) return fail(ADCT_ENOTSUP, "square roots of the row norms too large for the exact "
                                                        "decision of half ties");
    int64_t g = 1;
    while (g * g * r3 < p * q) ++g;
    int64_t D = 1;
    for (int i = 0; i < 64; ++i) {
        if ((i >> 3) + (i & 7) > band) continue;
        D = lcm64(D, mu[i] * rr[i]);
        if (D > (int64_t(1) << 40)) return fail(ADCT_ERANGE, "denominator of the exact half decision exceeds 2^40");
    }
    st->on = 1;
    st->p = int32_t(p);
    st->q = int32_t(q);
    st->g = int32_t(g);
    st->D = D;
    int tmax = 0;
    for (int i = 0; i < 64; ++i) tmax = std::max(tmax, std::abs(int(m.T[i])));
    for (int i = 0; i < 64; ++i) {
        const bool in = (i >> 3) + (i & 7) <= band;
        st->w[i] = in ? int32_t(D / (mu[i] * rr[i])) : 0;
        st->cls[i] = int8_t(rr[i] == 1 ? 0 : rr[i] == p ? 1 : rr[i] == q ? 2 : 3);
    }
    // every component of the sign test below 2^52 for |C| <= 32768, the pixel's
    // floor in [-1, 255]
    const __int128 cmax = 32768;
    __int128 nmax[4] = {0, 0, 0, 0};
    double sk = 0.0;
    for (int x = 0; x < 8; ++x)
        for (int y = 0; y < 8; ++y) {
            __int128 nb[4] = {0, 0, 0, 0};
            for (int k = 0; k < 8; ++k)
                for (int l = 0; l < 8; ++l) {
                    if (k + l > band) continue;
                    nb[st->cls[8 * k + l]] += cmax * std::abs(m.T[8 * k + x] * m.T[8 * l + y]) * st->w[8 * k + l];
                }
            for (int c = 0; c < 4; ++c) nmax[c] = std::max(nmax[c], nb[c]);
        }
    for (int i = 0; i < 64; ++i)
        if ((i >> 3) + (i & 7) <= band) sk += inv_sqrt_newton(int64_t(m.n[i >> 3]) * m.n[i & 7]);
    const __int128 s2 = 2 * __int128(step), lim = kSettleMaxComp;
    const __int128 comp[4] = {g * (s2 * nmax[0] + 513 * __int128(D)), g * s2 * nmax[1], g * s2 * nmax[2],
                              s2 * nmax[3]};
    for (int c = 0; c < 4; ++c)
        if (comp[c] >= lim) return fail(ADCT_ERANGE, "quant_step too large for the exact decision of half ties");
    // float64 error of a pixel below 20 2^-53 Tmax^2 step sum |C_kl| s_k s_l;
    // the tolerance is 8 times that, and must stay below 1/4 for any int16 levels
    st->tol_c = std::ldexp(1.0, -45) * double(tmax) * tmax * step;
    if (st->tol_c * 32768.0 * sk >= 0.25)
        return fail(ADCT_ERANGE, "quant_step too large for the exact decision of half ties");
    return ADCT_OK;
}

struct Prepared {
    adct_matrix m;
    int band;
    bool quant;
    bool runtime;      // the matrix goes to the run-time kernels (ADCT_CUSTOM, or a
                       // quantiser step whose halves need the exact decision)
    bool settle;       // the run-time kernels decide pixels near a half exactly
    RtMatArgs rt;
    QuantTables qt;    // built-in kernels' quantiser constants
};

// The exact bounds depend only on the matrix (and the prefix length) and the
// inverse one costs tens of microseconds of 128-bit arithmetic, more than a
// small image's kernel: each thread keeps the last few results, keyed by the
// matrix bytes and r, since a caller usually repeats one transform.
struct BoundEntry {
    bool valid = false;
    int8_t T[64];
    int32_t n[8];
    int r;                 // -1: only the forward bound is filled
    int64_t fwd, inv;
};
constexpr int kBoundSlots = 8;
static thread_local BoundEntry g_bounds[kBoundSlots];
static thread_local int g_bound_next = 0;

static BoundEntry *bound_lookup(const adct_matrix &m, int r) {
    for (BoundEntry &e : g_bounds)
        if (e.valid && (e.r == r || r < 0) && memcmp(e.T, m.T, sizeof(e.T)) == 0 && memcmp(e.n, m.n, sizeof(e.n)) == 0)
            return &e;
    return nullptr;
}

static int64_t fwd_bound_cached(const adct_matrix &m) {
    if (const BoundEntry *e = bound_lookup(m, -1)) return e->fwd;
    BoundEntry &e = g_bounds[g_bound_next];
    g_bound_next = (g_bound_next + 1) % kBoundSlots;
    e.valid = true;
    memcpy(e.T, m.T, sizeof(e.T));
    memcpy(e.n, m.n, sizeof(e.n));
    e.r = -1;
    e.fwd = fwd_bound(m);
    e.inv = 0;
    return e.fwd;
}

static int64_t inv_bound_cached(const adct_matrix &m, int r) {
    if (const BoundEntry *e = bound_lookup(m, r); e && e->r == r) return e->inv;
    BoundEntry &e = g_bounds[g_bound_next];
    g_bound_next = (g_bound_next + 1) % kBoundSlots;
    e.valid = true;
    memcpy(e.T, m.T, sizeof(e.T));
    memcpy(e.n, m.n, sizeof(e.n));
    e.r = r;
    e.fwd = fwd_bound(m);
    e.inv = inv_bound(m, r);
    return e.inv;
}

adct_status prepare(adct_transform_id t, const adct_matrix *custom, int r, int quant_step,
                    bool need_int16_coef, Prepared *out, CodecArgs *a) {
    if (t == ADCT_DCT) return fail(ADCT_ENOTSUP, "the exact DCT runs through the MFMA comparator path");
    if (t != ADCT_CUSTOM && !is_builtin_int(t)) return fail(ADCT_EINVAL, "unknown transform id");
    if (r < 1 || r > 64) return fail(ADCT_ERANGE, "r must be in [1, 64]");
    if (quant_step < 0 || quant_step > 65535) return fail(ADCT_ERANGE, "quant_step must be in [0, 65535]");
    out->runtime = (t == ADCT_CUSTOM);
    if (out->runtime) {
        adct_status st = check_custom(custom);
        if (st) return st;
        out->m = *custom;
    } else {
        matrix_of(t, &out->m);
    }
    out->band = r <= 10 ? 3 : 14;
    out->quant = quant_step > 0;
    // A dequantised reconstruction sum_kl T T step q / sqrt(n_k n_l) can sit
    // exactly on a half only through its rational part; that part has an odd
    // denominator (so never a half) when every perfect-square class mu^2 =
    // n_k n_l gives step / mu an odd reduced denominator.  Other steps go to the
    // run-time kernels, which decide pixels near a half exactly.
    out->settle = false;
    if (out->quant) {
        for (int k = 0; k < 8 && !out->settle; ++k)
            for (int l = 0; l < 8; ++l) {
                const int64_t prod = int64_t(out->m.n[k]) * out->m.n[l];
                const int64_t mu = int64_t(llround(sqrt(double(prod))));
                if (mu * mu != prod) continue;
                int64_t g = mu, b = quant_step;
                while (b) { const int64_t t2 = g % b; g = b; b = t2; }
                if (((mu / g) & 1) == 0) {
                    out->settle = true;
                    break;
                }
            }
        if (out->settle) out->runtime = true;
    }
    const int64_t fb = fwd_bound_cached(out->m);
    if (!out->quant) {
        if (need_int16_coef && fb > 32767)
            return fail(ADCT_EOVERFLOW, "the integer stage of this transform exceeds int16; request coef_scaled");
        if (out->runtime) {
            if (!rt_words_fit(out->m, std::max<int64_t>(fb, 32767)))
                return fail(ADCT_EOVERFLOW, "exact inverse of this matrix exceeds 64-bit words");
        } else if (2 * inv_bound_cached(out->m, r) + (int64_t(1) << 22) >= (int64_t(1) << 31)) {
            return fail(ADCT_EOVERFLOW, "inverse numerator exceeds int32");
        }
    } else if (out->runtime && fb >= kRtMaxQuantY) {
        return fail(ADCT_ERANGE, "custom matrix: |Y| bound too large for the float64 quantiser (>= 2^24)");
    }
    const int32_t *n = out->m.n;
    for (int k = 0; k < 8; ++k)
        for (int l = 0; l < 8; ++l) {
            const int64_t prod = int64_t(n[k]) * n[l];
            const int64_t mu = int64_t(llround(sqrt(double(prod))));
            if (out->quant && mu * mu == prod) {
                const int64_t d2 = 2 * int64_t(quant_step) * mu;
                if (2 * fb + d2 >= (int64_t(1) << 24) || d2 >= (int64_t(1) << 23))
                    return fail(ADCT_ERANGE, "quant_step too large for the exact integer quantiser");
                // the built-in kernels' float32 form (quant_rational_f) needs |Y| + d < 2^20
                if (!out->runtime && fb + d2 / 2 >= (int64_t(1) << 20))
                    return fail(ADCT_ERANGE, "quant_step too large for the exact quantiser");
            }
        }
    memset(&out->qt, 0, sizeof(out->qt));
    if (out->quant) {
        int32_t nn[8];
        for (int k = 0; k < 8; ++k) nn[k] = n[k];
        for (int k = 0; k < 8; ++k)
            for (int l = 0; l < 8; ++l) {
                const int c = class_of(nn, k, l);
                const int64_t prod = int64_t(n[k]) * n[l];
                const int64_t mu = int64_t(llround(sqrt(double(prod))));
                const double skl = inv_sqrt_newton(prod);
                const double d = double(quant_step) * double(mu);
                out->qt.qc1[c] = (mu * mu == prod) ? float(1.0 / d) : 0.f;
                out->qt.qc2[c] = (mu * mu == prod) ? float((d + 0.5) / (2.0 * d)) : 0.f;
                out->qt.qinv[c] = skl / double(quant_step);
                out->qt.qdeq[c] = double(quant_step) * skl;
            }
    }
    if (out->runtime) {
        adct_status st = build_rt(out->m, &out->rt);
        if (st) return st;
        if (out->settle) {
            st = build_settle(out->m, out->band, quant_step, &out->rt.st);
            if (st) return st;
        }
    }
    a->step = quant_step;
    a->inv_step_f = quant_step ? float(1.0 / quant_step) : 0.f;
    a->inv_step_d = quant_step ? 1.0 / quant_step : 0.0;
    a->step_d = double(quant_step);
    return ADCT_OK;
}

adct_status check_plane(const void *base, int64_t offset, int H, int W, int pitch, const char *what) {
    if (H <= 0 || W <= 0 || (H & 7) || (W & 7))
        return fail(ADCT_EDIM, std::string(what) + ": H and W must be positive multiples of 8");
    if (pitch < W) return fail(ADCT_EDIM, std::string(what) + ": pitch < W");
    if ((pitch & 7) || (offset & 7) || !aligned(base, 8))
        return fail(ADCT_EDIM, std::string(what) + ": base, offsets and pitch must be 8-byte aligned");
    if (int64_t(H / 8) * (W / 8) > (int64_t(1) << 30))
        return fail(ADCT_EDIM, std::string(what) + ": too many blocks");
    if (pitch >= (1 << 24) || H >= (1 << 24) || int64_t(H) * pitch >= (int64_t(1) << 32))
        return fail(ADCT_EDIM, std::string(what) + ": plane larger than 4 GiB, pitch >= 2^24 or H >= 2^24 "
                                                   "(row offsets are formed with 24-bit multiplies)");
    return ADCT_OK;
}

// Set up plane descriptors; returns waves per frame.
int setup_planes(CodecArgs *a, const adct_plane *pl, int np) {
    int waves = 0, blocks = 0;
    for (int p = 0; p < np; ++p) {
        PlaneArg &d = a->pl[p];
        d.in_off = pl[p].offset;
        d.out_off = pl[p].offset;
        d.pitch_in = pl[p].pitch;
        d.pitch_out = pl[p].pitch;
        d.nbx = pl[p].W / 8;
        d.nblocks = (pl[p].H / 8) * (pl[p].W / 8);
        d.wave_start = waves;
        d.block_off = blocks;
        magic_u31(uint32_t(d.nbx), &d.nbx_m, &d.nbx_s);
        waves += (d.nblocks + 63) / 64;
        blocks += d.nblocks;
    }
    a->n_planes = np;
    a->blocks_per_frame = blocks;
    a->waves_per_frame = waves;
    magic_u31(uint32_t(waves), &a->wpf_m, &a->wpf_s);
    return waves;
}

// Exact-DCT launch set-up: 16-block tiles per wave.
int setup_dct(DctArgs *a, const adct_plane *pl, int np, int r, int step) {
    int waves = 0, blocks = 0;
    for (int p = 0; p < np; ++p) {
        PlaneArg &d = a->pl[p];
        d.in_off = pl[p].offset;
        d.out_off = pl[p].offset;
        d.pitch_in = pl[p].pitch;
        d.pitch_out = pl[p].pitch;
        d.nbx = pl[p].W / 8;
        d.nblocks = (pl[p].H / 8) * (pl[p].W / 8);
        d.wave_start = waves;
        d.block_off = blocks;
        magic_u31(uint32_t(d.nbx), &d.nbx_m, &d.nbx_s);
        waves += (d.nblocks + 15) / 16;
        blocks += d.nblocks;
    }
    a->n_planes = np;
    a->blocks_per_frame = blocks;
    a->waves_per_frame = waves;
    magic_u31(uint32_t(waves), &a->wpf_m, &a->wpf_s);
    a->r = r;
    a->step = step;
    a->inv_step = step ? float(1.0 / step) : 0.f;
    for (int k = 0; k < 8; ++k)
        for (int x = 0; x < 8; ++x) {
            const double alpha = k == 0 ? sqrt(0.125) : 0.5;
            a->C[8 * k + x] = float(alpha * cos((2 * x + 1) * k * M_PI / 16.0));
        }
    return waves;
}

adct_status check_dct_args(int r, int quant_step) {
    if (r < 1 || r > 64) return fail(ADCT_ERANGE, "r must be in [1, 64]");
    if (quant_step < 0 || quant_step > 65535) return fail(ADCT_ERANGE, "quant_step must be in [0, 65535]");
    return ADCT_OK;
}

}  // namespace
}  // namespace adct

using namespace adct;

static adct_status stream_impl(const uint8_t *frames, int64_t frame_stride, int n_frames,
                               const adct_plane *planes, int n_planes,
                               adct_transform_id t, const adct_matrix *custom,
                               int r, int quant_step, int16_t *coef, uint8_t *recon,
                               int64_t frame_stride_out, int pitch_out_override,
                               uint64_t *sse, adct_stream_t stream) {
    if (!frames || !planes || !sse) return fail(ADCT_EINVAL, "frames, planes and sse are required");
    if (n_frames < 1) return fail(ADCT_ERANGE, "n_frames must be >= 1");
    if (n_planes < 1 || n_planes > kMaxPlanes) return fail(ADCT_ERANGE, "n_planes must be in [1, 4]");
    if (frame_stride < 0 || (frame_stride & 7)) return fail(ADCT_EDIM, "frame_stride must be a non-negative multiple of 8");
    if (recon && (frame_stride_out < 0 || (frame_stride_out & 7) || !aligned(recon, 8)))
        return fail(ADCT_EDIM, "recon must be 8-byte aligned with a frame stride multiple of 8");
    if (coef && !aligned(coef, 4)) return fail(ADCT_EDIM, "coef must be 4-byte aligned");
    if (!aligned(sse, 8)) return fail(ADCT_EDIM, "sse must be 8-byte aligned");
    for (int p = 0; p < n_planes; ++p) {
        adct_status st = check_plane(frames, planes[p].offset, planes[p].H, planes[p].W, planes[p].pitch, "plane");
        if (st) return st;
    }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    if (t == ADCT_DCT) {
        adct_status st = check_dct_args(r, quant_step);
        if (st) return st;
        if (coef && quant_step == 0)
            return fail(ADCT_EINVAL, "the exact DCT has integer output only with a quantiser step");
        DctArgs d;
        memset(&d, 0, sizeof(d));
        const int wpf = setup_dct(&d, planes, n_planes, r, quant_step);
        if (pitch_out_override > 0)
            for (int p = 0; p < n_planes; ++p) d.pl[p].pitch_out = pitch_out_override;
        if (int64_t(wpf) * n_frames >= (int64_t(1) << 31) / 4)
            return fail(ADCT_EDIM, "stream too large for one launch");
        d.in = frames;
        d.out = recon;
        d.coef_q = coef;
        d.sse = reinterpret_cast<unsigned long long *>(sse);
        d.fs_in = frame_stride;
        d.fs_out = frame_stride_out;
        d.n_frames = n_frames;
        st = zero_u64(sse, int64_t(n_frames) * n_planes, hs);
        if (st) return st;
        return launch_dct(kEvaluate, d, wpf * n_frames, hs);
    }
    CodecArgs a;
    memset(&a, 0, sizeof(a));
    Prepared pr;
    adct_status st = prepare(t, custom, r, quant_step, coef != nullptr, &pr, &a);
    if (st) return st;
    const int wpf = setup_planes(&a, planes, n_planes);
    if (pitch_out_override > 0)
        for (int p = 0; p < n_planes; ++p) a.pl[p].pitch_out = pitch_out_override;
    if (int64_t(wpf) * n_frames >= (int64_t(1) << 31) / 4)
        return fail(ADCT_EDIM, "stream too large for one launch");
    if (int64_t(a.blocks_per_frame) * n_frames * r >= (int64_t(1) << 62))
        return fail(ADCT_EDIM, "coefficient buffer too large");
    a.in = frames;
    a.out = recon;
    a.coef = coef;
    a.sse = reinterpret_cast<unsigned long long *>(sse);
    a.fs_in = frame_stride;
    a.fs_out = frame_stride_out;
    a.n_frames = n_frames;
    a.r = r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = zero_u64(sse, int64_t(n_frames) * n_planes, s);
    if (st) return st;
    if (pr.runtime) return launch_codec_rt(pr.band, pr.quant, false, kEvaluate, a, pr.rt, wpf * n_frames, s);
    return launch_codec(t, pr.band, pr.quant, kEvaluate, a, pr.qt, wpf * n_frames, s);
}

extern "C" {

adct_status adct_stream_bandwidth_probe(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                        const adct_plane *planes, int n_planes, int r, int16_t *coef,
                                        uint8_t *recon, int64_t frame_stride_out, adct_stream_t stream) {
    if (!frames || !planes) return fail(ADCT_EINVAL, "frames and planes are required");
    if (n_frames < 1) return fail(ADCT_ERANGE, "n_frames must be >= 1");
    if (n_planes < 1 || n_planes > kMaxPlanes) return fail(ADCT_ERANGE, "n_planes must be in [1, 4]");
    if (frame_stride < 0 || (frame_stride & 7)) return fail(ADCT_EDIM, "frame_stride must be a non-negative multiple of 8");
    if (recon && (frame_stride_out < 0 || (frame_stride_out & 7) || !aligned(recon, 8)))
        return fail(ADCT_EDIM, "recon must be 8-byte aligned with a frame stride multiple of 8");
    if (coef && !aligned(coef, 4)) return fail(ADCT_EDIM, "coef must be 4-byte aligned");
    for (int p = 0; p < n_planes; ++p) {
        adct_status st = check_plane(frames, planes[p].offset, planes[p].H, planes[p].W, planes[p].pitch, "plane");
        if (st) return st;
    }
    CodecArgs a;
    memset(&a, 0, sizeof(a));
    Prepared pr;
    adct_status st = prepare(ADCT_T1, nullptr, r, 0, false, &pr, &a);
    if (st) return st;
    const int wpf = setup_planes(&a, planes, n_planes);
    if (int64_t(wpf) * n_frames >= (int64_t(1) << 31) / 4) return fail(ADCT_EDIM, "stream too large for one launch");
    a.in = frames;
    a.out = recon;
    a.coef = coef;
    a.fs_in = frame_stride;
    a.fs_out = frame_stride_out;
    a.n_frames = n_frames;
    a.r = r;
    return launch_codec(ADCT_T1, pr.band, false, kProbe, a, pr.qt, wpf * n_frames, reinterpret_cast<hipStream_t>(stream));
}

const char *adct_last_error(void) { return g_err.c_str(); }

int adct_version(void) { return 100; }

adct_status adct_codec_set_schedule(int workgroups_per_cu) {
    if (workgroups_per_cu < -1 || workgroups_per_cu > 64)
        return fail(ADCT_ERANGE, "workgroups_per_cu must be in [-1, 64]");
    g_codec_wgs_per_cu = workgroups_per_cu;
    return ADCT_OK;
}

adct_status adct_release_caches(int64_t *bytes_released) {
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    const int64_t n = release_search_cache(dev) + release_gain_cache(dev);
    if (bytes_released) *bytes_released = n;
    return ADCT_OK;
}

adct_status adct_matrix_get(adct_transform_id id, adct_matrix *out) {
    if (!out) return fail(ADCT_EINVAL, "out is null");
    if (!is_builtin_int(id)) return fail(ADCT_EINVAL, "not a built-in integer transform");
    matrix_of(id, out);
    return ADCT_OK;
}

adct_status adct_check_codec_args(adct_transform_id t, const adct_matrix *custom, int r,
                                  int quant_step, int want_int16) {
    CodecArgs a;
    Prepared pr;
    return prepare(t, custom, r, quant_step, want_int16 != 0, &pr, &a);
}

adct_status adct_transform_bounds(adct_transform_id id, const adct_matrix *custom, int r,
                                  int quant_step, int64_t *fwd, int64_t *inv) {
    adct_matrix m;
    if (id == ADCT_CUSTOM) {
        if (!custom) return fail(ADCT_EINVAL, "custom matrix is null");
        m = *custom;
    } else if (is_builtin_int(id)) {
        matrix_of(id, &m);
    } else {
        return fail(ADCT_EINVAL, "not an integer transform");
    }
    if (r < 1 || r > 64) return fail(ADCT_ERANGE, "r must be in [1, 64]");
    if (quant_step < 0) return fail(ADCT_ERANGE, "quant_step < 0");
    for (int k = 0; k < 8; ++k)
        if (m.n[k] <= 0) return fail(ADCT_EINVAL, "matrix has a zero row");
    if (fwd) *fwd = fwd_bound_cached(m);
    if (inv) *inv = inv_bound_cached(m, r);
    return ADCT_OK;
}

adct_status adct_encode_blocks(const uint8_t *img, int H, int W, int pitch,
                               adct_transform_id t, const adct_matrix *custom,
                               int r, int quant_step, int16_t *coef_int, float *coef_scaled,
                               adct_stream_t stream) {
    if (!img) return fail(ADCT_EINVAL, "img is null");
    if (!coef_int && !coef_scaled) return fail(ADCT_EINVAL, "no output requested");
    adct_status st = check_plane(img, 0, H, W, pitch, "img");
    if (st) return st;
    if ((coef_int && !aligned(coef_int, 4)) || (coef_scaled && !aligned(coef_scaled, 4)))
        return fail(ADCT_EDIM, "coefficient buffers must be 4-byte aligned");
    if (t == ADCT_DCT) {
        st = check_dct_args(r, quant_step);
        if (st) return st;
        if (coef_int && quant_step == 0)
            return fail(ADCT_EINVAL, "the exact DCT has integer output only with a quantiser step");
        DctArgs d;
        memset(&d, 0, sizeof(d));
        adct_plane pl = {0, H, W, pitch, 0};
        const int waves = setup_dct(&d, &pl, 1, r, quant_step);
        d.in = img;
        d.coef_f = coef_scaled;
        d.coef_q = coef_int;
        d.n_frames = 1;
        return launch_dct(kEncode, d, waves, reinterpret_cast<hipStream_t>(stream));
    }
    CodecArgs a;
    memset(&a, 0, sizeof(a));
    Prepared pr;
    st = prepare(t, custom, r, quant_step, coef_int != nullptr, &pr, &a);
    if (st) return st;
    adct_plane pl = {0, H, W, pitch, 0};
    const int waves = setup_planes(&a, &pl, 1);
    a.in = img;
    a.coef = coef_int;
    a.coef_f = coef_scaled;
    a.n_frames = 1;
    a.r = r;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    if (pr.runtime) return launch_codec_rt(pr.band, pr.quant, false, kEncode, a, pr.rt, waves, hs);
    return launch_codec(t, pr.band, pr.quant, kEncode, a, pr.qt, waves, hs);
}

adct_status adct_decode_blocks(const int16_t *coef_int, const float *coef_scaled,
                               int H, int W, uint8_t *out, int pitch_out,
                               adct_transform_id t, const adct_matrix *custom,
                               int r, int quant_step, adct_stream_t stream) {
    if (!out) return fail(ADCT_EINVAL, "out is null");
    if ((coef_int != nullptr) == (coef_scaled != nullptr))
        return fail(ADCT_EINVAL, "exactly one of coef_int / coef_scaled must be given");
    adct_status st = check_plane(out, 0, H, W, pitch_out, "out");
    if (st) return st;
    if (t == ADCT_DCT) {
        st = check_dct_args(r, quant_step);
        if (st) return st;
        if (coef_int && quant_step == 0)
            return fail(ADCT_EINVAL, "integer DCT coefficients are quantised levels: give quant_step");
        if (coef_scaled && quant_step != 0)
            return fail(ADCT_EINVAL, "float DCT coefficients are decoded without a quantiser step");
        if (!aligned(coef_int ? (const void *)coef_int : (const void *)coef_scaled, 4))
            return fail(ADCT_EDIM, "coefficients must be 4-byte aligned");
        DctArgs d;
        memset(&d, 0, sizeof(d));
        adct_plane pl = {0, H, W, pitch_out, 0};
        const int waves = setup_dct(&d, &pl, 1, r, quant_step);
        d.out = out;
        d.coef_f = const_cast<float *>(coef_scaled);
        d.coef_q = const_cast<int16_t *>(coef_int);
        d.n_frames = 1;
        return launch_dct(kDecode, d, waves, reinterpret_cast<hipStream_t>(stream));
    }
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    if (!aligned(coef_int ? (const void *)coef_int : (const void *)coef_scaled, 4))
        return fail(ADCT_EDIM, "coefficients must be 4-byte aligned");
    CodecArgs a;
    memset(&a, 0, sizeof(a));
    Prepared pr;
    adct_plane pl = {0, H, W, pitch_out, 0};
    if (coef_scaled) {
        // float B: A = C_hat^T B' C_hat in float64 with the run-time kernel
        if (quant_step != 0)
            return fail(ADCT_EINVAL, "float coefficients are decoded without a quantiser step");
        st = prepare(t, custom, r, 0, false, &pr, &a);
        if (st) return st;
        st = build_rt(pr.m, &pr.rt);
        if (st) return st;
        const int waves = setup_planes(&a, &pl, 1);
        a.out = out;
        a.coef_f = const_cast<float *>(coef_scaled);
        a.n_frames = 1;
        a.r = r;
        return launch_codec_rt(pr.band, false, true, kDecode, a, pr.rt, waves, hs);
    }
    st = prepare(t, custom, r, quant_step, true, &pr, &a);
    if (st) return st;
    const int waves = setup_planes(&a, &pl, 1);
    a.out = out;
    a.coef = const_cast<int16_t *>(coef_int);
    a.n_frames = 1;
    a.r = r;
    if (pr.runtime) return launch_codec_rt(pr.band, pr.quant, false, kDecode, a, pr.rt, waves, hs);
    return launch_codec(t, pr.band, pr.quant, kDecode, a, pr.qt, waves, hs);
}

adct_status adct_evaluate_stream(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                 const adct_plane *planes, int n_planes,
                                 adct_transform_id t, const adct_matrix *custom,
                                 int r, int quant_step, int16_t *coef, uint8_t *recon,
                                 int64_t frame_stride_out, uint64_t *sse, adct_stream_t stream) {
    return stream_impl(frames, frame_stride, n_frames, planes, n_planes, t, custom, r, quant_step,
                       coef, recon, frame_stride_out, 0, sse, stream);
}

adct_status adct_evaluate_coding(const uint8_t *img, int H, int W, int pitch,
                                 adct_transform_id t, const adct_matrix *custom,
                                 int r, int quant_step, int16_t *coef_int, uint8_t *recon,
                                 int pitch_out, uint64_t *sse_dev, double *mse_host,
                                 double *psnr_host, adct_stream_t stream) {
    if (!img || !sse_dev) return fail(ADCT_EINVAL, "img and sse_dev are required");
    adct_status st = check_plane(img, 0, H, W, pitch, "img");
    if (st) return st;
    if (recon) {
        st = check_plane(recon, 0, H, W, pitch_out, "recon");
        if (st) return st;
    }
    adct_plane pl = {0, H, W, pitch, 0};
    st = stream_impl(img, 0, 1, &pl, 1, t, custom, r, quant_step, coef_int, recon, 0,
                     recon ? pitch_out : 0, sse_dev, stream);
    if (st) return st;
    if (mse_host || psnr_host) {
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        uint64_t h = 0;
        ADCT_HIP(hipMemcpyAsync(&h, sse_dev, sizeof(h), hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipStreamSynchronize(s));
        const double mse = double(h) / (double(H) * double(W));
        if (mse_host) *mse_host = mse;
        if (psnr_host) *psnr_host = (h == 0) ? INFINITY : 10.0 * log10(255.0 * 255.0 / mse);
    }
    return ADCT_OK;
}

}  // extern "C"
