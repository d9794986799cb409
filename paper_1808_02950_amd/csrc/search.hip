// Angle-similarity search for low-complexity DCT rows (Sec. 3 and Sec. 4.1 of
// the paper), batched on the GPU.
//
// The search space D = P^8 (Sec. 3.2) is enumerated once into a device table
// (packed int8 vectors, primitive flags); a candidate's cosine to
// a DCT row is recomputed where it is needed (one float64 dot product of eight
// terms and the candidate's inverse norm: cheaper than reading 64 bytes of
// stored cosines per candidate, and always the same value).  The
// greedy problem of Eq. (6) is then answered query by query: a query is (rows
// already chosen, DCT row to approximate); the device finds the largest cosine
// (smallest angle, Sec. 3.3) among candidates orthogonal to every chosen row
// (Sec. 3.4) and collects every candidate within a small window of it; the host
// groups exact ties and expands the search tree level by level, so each launch
// answers every open query of one depth.
//
// The top-k form scans the whole space once per row with a per-workgroup LDS
// histogram of the angle, picks a cosine threshold per row, collects the
// candidates above it and ranks them on the host.  Orthogonal 8-tuples of the
// ranked lists are found by a depth-first search over orthogonality bitsets the
// device computes.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr double kTieEps = 1e-12;     // cosines this close are an exact tie in reals
constexpr double kWindow = 1e-6;      // collection window below the best cosine
constexpr int kHistBins = 448;        // 8 bins per octave of 1 - cos, 56 octaves

struct DctRows {
    double c[64];                     // orthonormal DCT-II rows, c[8k + n]
};

// The digit values in canonical order, 5 bits each (value + 16), and the
// reciprocal for dividing canonical indices by the base: for idx < 2^28 and a
// base b <= 9, umulhi(idx, ceil(2^32 / b)) is the exact quotient.
struct Digits {
    unsigned long long packed;
    unsigned long long primes;   // 4 bits per digit: value odd, not a multiple of 3, of 5, of 7
    uint32_t magic;
};

DctRows dct_rows() {
    DctRows r;
    for (int k = 0; k < 8; ++k)
        for (int x = 0; x < 8; ++x)
            r.c[8 * k + x] = (k == 0 ? sqrt(0.125) : 0.5) * cos((2 * x + 1) * k * M_PI / 16.0);
    return r;
}

__device__ __forceinline__ int sdot8(uint2 a, uint2 b) {
    return __builtin_amdgcn_sdot4(int(a.x), int(b.x), __builtin_amdgcn_sdot4(int(a.y), int(b.y), 0, false),
                                  false);
}

__device__ __forceinline__ void unpack8(uint2 p, int (&v)[8]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] = int(int8_t(uint8_t(p.x >> (8 * e))));
        v[4 + e] = int(int8_t(uint8_t(p.y >> (8 * e))));
    }
}

// 1 / |v| in float64 (|v|^2 is an exact integer)
// (|v|^2 is an exact integer, at most 8 * 64: a table of 1 / sqrt(n) for every
// n replaces the square root and division in the scans; k_inv_table fills it
// with the same float64 expression)
constexpr int kMaxNorm2 = 512;
__device__ __forceinline__ double inv_norm(uint2 p, const double *invt) { return invt[sdot8(p, p)]; }

__global__ void k_inv_table(double *t) {
    const int n = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (n <= kMaxNorm2) t[n] = n ? 1.0 / sqrt(double(n)) : 0.0;
}

// cos of the angle between v and DCT row r: the float64 dot product in entry
// order, times 1 / |v| (the DCT rows have unit norm)
__device__ __forceinline__ double cos_row(const int (&v)[8], double inv, const DctRows &rows, int r) {
    double dot = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) dot = fma(double(v[e]), rows.c[8 * r + e], dot);
    return dot * inv;
}

// The same product with the rows read from LDS.  The scan kernels over the whole
// space keep all 64 entries there: as a kernel argument they are 128 scalar
// registers, more than a wave holds beside the rest, and the compiler reloads
// the spilled ones lane by lane for every candidate.
__device__ __forceinline__ double cos_row_lds(const int (&v)[8], double inv, const double *c, int r) {
    double dot = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) dot = fma(double(v[e]), c[8 * r + e], dot);
    return dot * inv;
}

// the rows into a workgroup's LDS copy (every thread calls it, before any use)
__device__ __forceinline__ void rows_to_lds(const DctRows &rows, double *sc) {
    for (int i = int(threadIdx.x); i < 64; i += int(blockDim.x)) sc[i] = rows.c[i];
}
// at the top of each candidate: the rows are read from LDS where they are used
// (a compiler-only barrier; without it the compiler would hoist all 64 into
// 128 vector registers)
__device__ __forceinline__ void rows_fence() { asm volatile("" ::: "memory"); }

// monotone map of a double onto uint64 (for atomicMax)
__device__ __forceinline__ unsigned long long order_key(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double key_value(unsigned long long k) {
    const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __builtin_bit_cast(double, u);
}

// ------------------------------------------------------------ enumeration

__global__ void k_enum(int b, Digits dg, int64_t n, uint2 *vec, uint8_t *prim) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t idx = uint32_t(i + 1);                  // canonical index; 0 is the zero vector
    int v[8];
    uint32_t dig[8];
#pragma unroll
    for (int e = 7; e >= 0; --e) {                   // first coordinate most significant
        const uint32_t q = __umulhi(idx, dg.magic);
        const uint32_t d = idx - q * uint32_t(b);
        dig[e] = d;
        v[e] = int((dg.packed >> (5 * d)) & 31u) - 16;
        idx = q;
    }
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t byte = uint32_t(uint8_t(int8_t(v[e])));
        if (e < 4) lo |= byte << (8 * e); else hi |= byte << (8 * (e - 4));
    }
    vec[i] = make_uint2(lo, hi);
    // gcd of the entries is 1 exactly when no prime divides all of them; the
    // entries are within +-8, so only 2, 3, 5 and 7 can: OR the digits'
    // "not divisible" bits and require all four
    uint32_t nd = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) nd |= uint32_t(dg.primes >> (4 * dig[e])) & 15u;
    prim[i] = uint8_t(nd == 15u);
}

// ------------------------------------------------------------ greedy queries

// A query: DCT row `row` against the candidates of one feasible list (the
// candidates orthogonal to every row chosen so far, as space indices).
struct Query {
    int64_t off;          // first entry of the list in the level's list arena
    int32_t len;
    int32_t row;
};

__global__ __launch_bounds__(256) void k_qmax(const Query *qs, const uint32_t *lists, const uint2 *vec,
                                             const double *invt, const DctRows rows, unsigned long long *best) {
    const Query q = qs[blockIdx.y];
    double m = -2.0;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < q.len;
         t += int64_t(gridDim.x) * blockDim.x) {
        const uint2 p = vec[lists[q.off + t]];
        int v[8];
        unpack8(p, v);
        m = fmax(m, cos_row(v, inv_norm(p, invt), rows, q.row));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > -2.0) atomicMax(best + blockIdx.y, order_key(m));
}

__global__ __launch_bounds__(256) void k_qcollect(const Query *qs, const uint32_t *lists, const uint2 *vec,
                                                 const double *invt, const DctRows rows,
                                                 const unsigned long long *best,
                                                 int cap, int64_t *out_idx, double *out_cos,
                                                 int *count) {
    const int qi = blockIdx.y;
    if (best[qi] == 0) return;                                  // no feasible candidate
    const Query q = qs[qi];
    const double lo = key_value(best[qi]) - kWindow;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < q.len;
         t += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t i = lists[q.off + t];
        const uint2 p = vec[i];
        int v[8];
        unpack8(p, v);
        const double c = cos_row(v, inv_norm(p, invt), rows, q.row);
        if (c >= lo) {
            const int pos = atomicAdd(count + qi, 1);
            if (pos < cap) {
                out_idx[int64_t(qi) * cap + pos] = int64_t(i);
                out_cos[int64_t(qi) * cap + pos] = c;
            }
        }
    }
}

// Feasible lists.  The root list holds every candidate orthogonal to the fixed
// rows; a child state's list keeps the parent's entries orthogonal to the
// candidate just chosen (the chosen one itself drops out: |v|^2 > 0).  Entry
// order inside a list follows the atomics and does not matter: the queries take
// a maximum and a window, and the host orders what they collect.
// Append for a whole wave with one atomic: the lanes that keep an entry take
// consecutive slots after the wave's base (ballot, popcount, lane prefix).  Every
// lane of the wave calls it.
__device__ __forceinline__ int64_t wave_append(int *counter, bool keep) {
    const unsigned long long mask = __ballot(keep);
    if (!mask) return -1;
    const int lane = int(threadIdx.x & 63);
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader, 64);
    return keep ? int64_t(base) + __popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

// the loops run a wave-uniform number of rounds so every lane reaches the ballot
__global__ __launch_bounds__(256) void k_root_list(int64_t n, const uint2 *vec, uint2 f0, uint2 f1, int nfixed,
                                                  uint32_t *out, int *len) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t first = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
    for (int64_t w = first; w < n; w += stride) {
        const int64_t i = w + (threadIdx.x & 63);
        bool ok = i < n;
        if (ok) {
            const uint2 p = vec[i];
            if (nfixed > 0) ok &= sdot8(p, f0) == 0;
            if (nfixed > 1) ok &= sdot8(p, f1) == 0;
        }
        const int64_t pos = wave_append(len, ok);
        if (ok) out[pos] = uint32_t(i);
    }
}

struct FilterJob {
    int64_t in_off, out_off;
    int32_t in_len;
    uint32_t chosen;      // space index of the candidate just chosen
};

__global__ __launch_bounds__(256) void k_filter(const uint2 *vec, const uint32_t *in, const FilterJob *jobs,
                                               uint32_t *out, int *lens) {
    const FilterJob j = jobs[blockIdx.y];
    const uint2 c = vec[j.chosen];
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t first = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
    for (int64_t w = first; w < j.in_len; w += stride) {
        const int64_t t = w + (threadIdx.x & 63);
        uint32_t i = 0;
        bool keep = t < j.in_len;
        if (keep) {
            i = in[j.in_off + t];
            keep = sdot8(vec[i], c) == 0;
        }
        const int64_t pos = wave_append(lens + blockIdx.y, keep);
        if (keep) out[j.out_off + pos] = i;
    }
}

// ------------------------------------------------------------ top-k scan

// Bins of the angle histogram: 8 per octave of u = 1 - cos, read off the float64
// representation of u: its biased exponent E and the top three fraction bits
// t give key = 8 E + t, monotone in u, and bin = 8183 - key runs 0..7 over
// [1/2, 1), 8..15 over [1/4, 1/2), and so on (u >= 1, angles of 90 degrees or
// more, gives a negative bin, which is not counted).  The histogram and the
// collection use the same bins, and the host ranks the collected candidates
// exactly, so the edges need only be fixed and monotone.  c >= 1 is the last bin.
__device__ __forceinline__ int angle_bin(double c) {
    const double u = 1.0 - c;
    if (!(u > 0.0)) return kHistBins - 1;
    const uint32_t hi = uint32_t((unsigned long long)__double_as_longlong(u) >> 32);
    const int b = 8183 - int(hi >> 17);
    return b >= kHistBins ? kHistBins - 1 : b;
}

// The histogram pass also leaves each candidate's eight bins as bytes (bin + 1
// clamped to [0, 255]; 0 for a skipped candidate or an angle of 90 degrees or
// more), so the collection pass compares bytes and computes cosines only for
// the few candidates it keeps.
__global__ __launch_bounds__(256) void k_hist(int64_t n, const uint2 *vec, const uint8_t *prim, int primitive,
                                             const double *invt, const DctRows rows, unsigned *hist,
                                             uint2 *codes) {
    __shared__ unsigned h[8 * kHistBins];
    __shared__ double sc[64];
    for (int i = threadIdx.x; i < 8 * kHistBins; i += blockDim.x) h[i] = 0;
    rows_to_lds(rows, sc);
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        rows_fence();
        uint32_t c0 = 0, c1 = 0;
        if (!(primitive && !prim[i])) {
            const uint2 p = vec[i];
            int v[8];
            unpack8(p, v);
            const double inv = inv_norm(p, invt);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int bn = angle_bin(cos_row_lds(v, inv, sc, r));
                if (bn >= 0) atomicAdd(&h[r * kHistBins + bn], 1u);
                const uint32_t code = uint32_t(min(max(bn + 1, 0), 255));
                if (r < 4) c0 |= code << (8 * r); else c1 |= code << (8 * (r - 4));
            }
        }
        codes[i] = make_uint2(c0, c1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * kHistBins; i += blockDim.x)
        if (h[i]) atomicAdd(hist + i, h[i]);
}

struct Thresholds {
    int bin[8];                                                 // collect bins >= bin[r]
    int64_t cap[8];
    int64_t off[8];
};

__global__ __launch_bounds__(256) void k_topk_collect(int64_t n, const uint2 *vec, const uint8_t *prim,
                                                     int primitive, const double *invt, const DctRows rows,
                                                     Thresholds th,
                                                     int64_t *out_idx, double *out_cos,
                                                     unsigned long long *count) {
    __shared__ double sc[64];
    rows_to_lds(rows, sc);
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        rows_fence();
        if (primitive && !prim[i]) continue;
        const uint2 p = vec[i];
        int v[8];
        unpack8(p, v);
        const double inv = inv_norm(p, invt);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const double c = cos_row_lds(v, inv, sc, r);
            if (angle_bin(c) >= th.bin[r]) {
                const unsigned long long pos = atomicAdd(count + r, 1ull);
                if (int64_t(pos) < th.cap[r]) {
                    out_idx[th.off[r] + int64_t(pos)] = i;
                    out_cos[th.off[r] + int64_t(pos)] = c;
                }
            }
        }
    }
}

// Collection from the stored bins: a candidate joins row r's list when its byte
// reaches th.bin[r] + 1 (the same test as angle_bin >= th.bin[r] while
// th.bin[r] <= 254; the host uses the recomputing kernel otherwise).
__global__ __launch_bounds__(256) void k_topk_collect_codes(int64_t n, const uint2 *codes, const uint2 *vec,
                                                           const double *invt, const DctRows rows,
                                                           Thresholds th, int64_t *out_idx, double *out_cos,
                                                           unsigned long long *count) {
    __shared__ double sc[64];
    rows_to_lds(rows, sc);
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        rows_fence();
        const uint2 cw = codes[i];
        uint32_t hit = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int code = int(((r < 4 ? cw.x : cw.y) >> (8 * (r & 3))) & 0xffu);
            hit |= (code >= th.bin[r] + 1) ? (1u << r) : 0u;
        }
        if (!hit) continue;
        const uint2 p = vec[i];
        int v[8];
        unpack8(p, v);
        const double inv = inv_norm(p, invt);
        for (int r = 0; r < 8; ++r) {
            if (!((hit >> r) & 1u)) continue;
            const unsigned long long pos = atomicAdd(count + r, 1ull);
            if (int64_t(pos) < th.cap[r]) {
                out_idx[th.off[r] + int64_t(pos)] = i;
                out_cos[th.off[r] + int64_t(pos)] = cos_row_lds(v, inv, sc, r);
            }
        }
    }
}

// ------------------------------------------------------------ orthogonality bitsets

// bits[(pair * kmax + a) * words + w] bit j: lists[r1][a] . lists[r2][64 w + j] == 0
__global__ void k_ortho_bits(const uint2 *lists, const int *len, const int *base, int kmax, int words,
                             unsigned long long *bits) {
    const int pair = blockIdx.y;
    int r1 = 0, rem = pair;
    while (rem >= 7 - r1) {
        rem -= 7 - r1;
        ++r1;
    }
    const int r2 = r1 + 1 + rem;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int a = int(t / words), w = int(t % words);
    if (a >= len[r1]) return;
    const uint2 va = lists[base[r1] + a];
    unsigned long long word = 0;
    for (int j = 0; j < 64; ++j) {
        const int q = 64 * w + j;
        if (q < len[r2] && sdot8(va, lists[base[r2] + q]) == 0) word |= 1ull << j;
    }
    bits[(int64_t(pair) * kmax + a) * words + w] = word;
}

// ------------------------------------------------------------ host helpers

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

template <class T>
adct_status dalloc(DevBuf &b, size_t count) {
    ADCT_HIP(hipMalloc(&b.p, std::max<size_t>(count, 1) * sizeof(T)));
    return ADCT_OK;
}

// Device buffers the searches reuse from call to call (the enumerated space,
// its primitive flags, the top-k bin codes): grow-only, per device, kept until
// the process ends.  A search holds its device's lock from the space's
// enumeration until it has synchronised its stream and returned, so searches on
// one device run one at a time.
// slots: 0 space, 1 primitive flags, 2 top-k bin bytes, 3-7 closure queries,
// maxima, counts, collected indices and cosines, 8-9 feasible-list arenas of
// two consecutive depths, 10-11 filter jobs and list lengths
constexpr int kCacheSlots = 12;
struct SearchCache {
    std::mutex lock;
    void *slot[kCacheSlots] = {};
    size_t bytes[kCacheSlots] = {};
};
constexpr int kCacheDevices = 64;
SearchCache g_cache[kCacheDevices];

}  // namespace

// free the current device's search buffers (waits for a running search on it)
int64_t release_search_cache(int dev) {
    if (dev < 0 || dev >= kCacheDevices) return 0;
    SearchCache &c = g_cache[dev];
    std::lock_guard<std::mutex> hold(c.lock);
    int64_t n = 0;
    for (int i = 0; i < kCacheSlots; ++i) {
        if (c.slot[i]) (void)hipFree(c.slot[i]);
        n += int64_t(c.bytes[i]);
        c.slot[i] = nullptr;
        c.bytes[i] = 0;
    }
    return n;
}

namespace {

struct Space {
    int b = 0;
    int8_t digits[9] = {};
    int64_t n = 0;
    std::unique_lock<std::mutex> hold;    // the device's cache, for the whole search
    SearchCache *cache = nullptr;
    void *vec = nullptr, *prim = nullptr;
    DevBuf inv;
};

adct_status cached(Space &sp, int slot, size_t bytes, void **out);
template <class T>
adct_status cached_n(Space &sp, int slot, int64_t count, T **out) {
    void *p = nullptr;
    adct_status st = cached(sp, slot, size_t(std::max<int64_t>(count, 1)) * sizeof(T), &p);
    *out = static_cast<T *>(p);
    return st;
}

// buffer `slot` of the held cache with at least `bytes` bytes
adct_status cached(Space &sp, int slot, size_t bytes, void **out) {
    SearchCache &c = *sp.cache;
    if (c.bytes[slot] < bytes) {
        if (c.slot[slot]) ADCT_HIP(hipFree(c.slot[slot]));
        c.slot[slot] = nullptr;
        c.bytes[slot] = 0;
        ADCT_HIP(hipMalloc(&c.slot[slot], bytes));
        c.bytes[slot] = bytes;
    }
    *out = c.slot[slot];
    return ADCT_OK;
}

adct_status canonical_digits(const int8_t *P, int nP, int8_t *out, int *b) {
    if (!P) return fail(ADCT_EINVAL, "P is null");
    if (nP < 1 || nP > 9) return fail(ADCT_ERANGE, "|P| must be in [1, 9]");
    std::vector<int> v(P, P + nP);
    std::sort(v.begin(), v.end());
    if (std::unique(v.begin(), v.end()) != v.end()) return fail(ADCT_EINVAL, "P has repeated entries");
    for (int x : v)
        if (x < -8 || x > 8) return fail(ADCT_ERANGE, "entries of P must be within [-8, 8]");
    // order 0, 1, -1, 2, -2, ... (the canonical index's digit order)
    std::sort(v.begin(), v.end(), [](int a, int c) {
        const int aa = a < 0 ? -a : a, cc = c < 0 ? -c : c;
        return aa != cc ? aa < cc : (a > c);
    });
    if (v[0] != 0) return fail(ADCT_EINVAL, "P must contain 0");
    for (int i = 0; i < nP; ++i) out[i] = int8_t(v[i]);
    *b = nP;
    return ADCT_OK;
}

adct_status build_space(const int8_t *P, int nP, Space &sp, hipStream_t s) {
    adct_status st = canonical_digits(P, nP, sp.digits, &sp.b);
    if (st) return st;
    int64_t total = 1;
    for (int i = 0; i < 8; ++i) total *= sp.b;
    sp.n = total - 1;
    if (sp.n < 1) return fail(ADCT_ERANGE, "search space is empty");
    int dev = 0;
    ADCT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kCacheDevices) return fail(ADCT_ENOTSUP, "device index beyond the search cache");
    sp.cache = &g_cache[dev];
    sp.hold = std::unique_lock<std::mutex>(sp.cache->lock);
    if ((st = cached(sp, 0, size_t(sp.n) * sizeof(uint2), &sp.vec))) return st;
    if ((st = cached(sp, 1, size_t(sp.n), &sp.prim))) return st;
    Digits dg;
    dg.packed = 0;
    dg.primes = 0;
    for (int i = 0; i < sp.b; ++i) {
        const int v = sp.digits[i];
        dg.packed |= (unsigned long long)(v + 16) << (5 * i);
        const unsigned long long m = (v % 2 != 0 ? 1u : 0u) | (v % 3 != 0 ? 2u : 0u) | (v % 5 != 0 ? 4u : 0u) |
                                     (v % 7 != 0 ? 8u : 0u);
        dg.primes |= m << (4 * i);
    }
    dg.magic = uint32_t(((uint64_t(1) << 32) + uint64_t(sp.b) - 1) / uint64_t(sp.b));   // ceil(2^32 / b)
    if (sp.b == 1) dg.magic = 0xffffffffu;           // b = 1 never divides (only the zero vector)
    const int64_t blocks = (sp.n + 255) / 256;
    hipLaunchKernelGGL(k_enum, dim3(unsigned(blocks)), dim3(256), 0, s, sp.b, dg, sp.n,
                       (uint2 *)sp.vec, (uint8_t *)sp.prim);
    ADCT_HIP(hipGetLastError());
    if ((st = dalloc<double>(sp.inv, kMaxNorm2 + 1))) return st;
    hipLaunchKernelGGL(k_inv_table, dim3((kMaxNorm2 + 256) / 256), dim3(256), 0, s, (double *)sp.inv.p);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}

// vector of canonical index idx (>= 1) as 8 int8 entries
void decode_index(const Space &sp, int64_t idx, int8_t *v) {
    for (int e = 7; e >= 0; --e) {
        v[e] = sp.digits[idx % sp.b];
        idx /= sp.b;
    }
}

uint2 pack8(const int8_t *v) {
    uint32_t lo = 0, hi = 0;
    for (int e = 0; e < 4; ++e) lo |= uint32_t(uint8_t(v[e])) << (8 * e);
    for (int e = 0; e < 4; ++e) hi |= uint32_t(uint8_t(v[4 + e])) << (8 * e);
    return make_uint2(lo, hi);
}

int norm2_of(const int8_t *v) {
    int s = 0;
    for (int e = 0; e < 8; ++e) s += v[e] * v[e];
    return s;
}

struct Cand {
    int64_t idx;    // canonical index
    double cos;
    int norm2;
};

// best tie group of a collected window: sort by cosine (descending, then index),
// extend from the top while consecutive cosines differ by at most kTieEps
std::vector<Cand> top_group(std::vector<Cand> c) {
    std::sort(c.begin(), c.end(), [](const Cand &a, const Cand &b) {
        return a.cos != b.cos ? a.cos > b.cos : a.idx < b.idx;
    });
    size_t k = c.empty() ? 0 : 1;
    while (k < c.size() && c[k - 1].cos - c[k].cos <= kTieEps) ++k;
    c.resize(k);
    return c;
}

// canonical rank: tie groups of cosine (single linkage on the sorted values),
// then smaller squared norm, then smaller index
void canonical_sort(std::vector<Cand> &c) {
    std::sort(c.begin(), c.end(), [](const Cand &a, const Cand &b) {
        return a.cos != b.cos ? a.cos > b.cos : a.idx < b.idx;
    });
    std::vector<int> grp(c.size(), 0);
    for (size_t i = 1; i < c.size(); ++i) grp[i] = grp[i - 1] + (c[i - 1].cos - c[i].cos > kTieEps ? 1 : 0);
    std::vector<size_t> ord(c.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
        if (grp[a] != grp[b]) return grp[a] < grp[b];
        if (c[a].norm2 != c[b].norm2) return c[a].norm2 < c[b].norm2;
        return c[a].idx < c[b].idx;
    });
    std::vector<Cand> out;
    out.reserve(c.size());
    for (size_t i : ord) out.push_back(c[i]);
    c.swap(out);
}

// prefix tree of row orders
struct Tree {
    std::vector<std::map<int, int>> kids;
    std::vector<int64_t> leaves;          // orders ending under each node
    int add_node() {
        kids.emplace_back();
        leaves.push_back(0);
        return int(kids.size()) - 1;
    }
};

struct State {
    int node;
    int8_t rows[8][8];
    bool set[8];
    int64_t loff;         // the state's feasible list in the current level's arena
    int32_t llen;
    uint32_t chosen;      // space index of the candidate chosen last (for the child list)
};

struct MatKey {
    std::array<uint8_t, 64> b;
    bool operator<(const MatKey &o) const { return memcmp(b.data(), o.b.data(), 64) < 0; }
};

// Answer a batch of queries: per query the collected window (or none when the
// feasible set is empty).
adct_status run_queries(Space &sp, const uint32_t *lists, const std::vector<Query> &qs,
                        std::vector<std::vector<Cand>> &res, std::vector<char> &dead, hipStream_t s) {
    const int nq = int(qs.size());
    res.assign(nq, {});
    dead.assign(nq, 0);
    if (nq == 0) return ADCT_OK;
    int cap = 64;
    Query *dq_p = nullptr;
    unsigned long long *dbest_p = nullptr;
    int *dcount_p = nullptr;
    adct_status st;
    if ((st = cached_n(sp, 3, nq, &dq_p))) return st;
    if ((st = cached_n(sp, 4, nq, &dbest_p))) return st;
    if ((st = cached_n(sp, 5, nq, &dcount_p))) return st;
    ADCT_HIP(hipMemcpyAsync(dq_p, qs.data(), sizeof(Query) * nq, hipMemcpyHostToDevice, s));
    ADCT_HIP(hipMemsetAsync(dbest_p, 0, sizeof(unsigned long long) * nq, s));
    int64_t maxlen = 1;
    for (const Query &q : qs) maxlen = std::max<int64_t>(maxlen, q.len);
    const unsigned chunks = unsigned(std::min<int64_t>((maxlen + 255) / 256, 64));
    for (int y0 = 0; y0 < nq; y0 += 65535) {
        const int ny = std::min(nq - y0, 65535);
        hipLaunchKernelGGL(k_qmax, dim3(chunks, ny), dim3(256), 0, s, dq_p + y0, lists,
                           (const uint2 *)sp.vec, (const double *)sp.inv.p, dct_rows(),
                           dbest_p + y0);
        ADCT_HIP(hipGetLastError());
    }
    for (;;) {
        int64_t *didx_p = nullptr;
        double *dcos_p = nullptr;
        if ((st = cached_n(sp, 6, int64_t(nq) * cap, &didx_p))) return st;
        if ((st = cached_n(sp, 7, int64_t(nq) * cap, &dcos_p))) return st;
        ADCT_HIP(hipMemsetAsync(dcount_p, 0, sizeof(int) * nq, s));
        for (int y0 = 0; y0 < nq; y0 += 65535) {
            const int ny = std::min(nq - y0, 65535);
            hipLaunchKernelGGL(k_qcollect, dim3(chunks, ny), dim3(256), 0, s, dq_p + y0,
                               lists, (const uint2 *)sp.vec, (const double *)sp.inv.p, dct_rows(),
                               dbest_p + y0, cap,
                               didx_p + int64_t(y0) * cap, dcos_p + int64_t(y0) * cap,
                               dcount_p + y0);
            ADCT_HIP(hipGetLastError());
        }
        std::vector<int> cnt(nq);
        std::vector<unsigned long long> best(nq);
        ADCT_HIP(hipMemcpyAsync(cnt.data(), dcount_p, sizeof(int) * nq, hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipMemcpyAsync(best.data(), dbest_p, sizeof(unsigned long long) * nq, hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipStreamSynchronize(s));
        const int need = *std::max_element(cnt.begin(), cnt.end());
        if (need > cap) {                    // window larger than the buffer: grow and redo
            cap = need;
            continue;
        }
        std::vector<int64_t> idx(int64_t(nq) * cap);
        std::vector<double> cs(int64_t(nq) * cap);
        ADCT_HIP(hipMemcpyAsync(idx.data(), didx_p, sizeof(int64_t) * idx.size(), hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipMemcpyAsync(cs.data(), dcos_p, sizeof(double) * cs.size(), hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < nq; ++q) {
            if (best[q] == 0) {
                dead[q] = 1;
                continue;
            }
            for (int j = 0; j < cnt[q]; ++j) {
                Cand c;
                c.idx = idx[int64_t(q) * cap + j] + 1;
                c.cos = cs[int64_t(q) * cap + j];
                int8_t v[8];
                decode_index(sp, c.idx, v);
                c.norm2 = norm2_of(v);
                res[q].push_back(c);
            }
        }
        return ADCT_OK;
    }
}

void fill_matrix(const int8_t (*rows)[8], adct_matrix *m) {
    for (int k = 0; k < 8; ++k) {
        int32_t s = 0;
        for (int e = 0; e < 8; ++e) {
            m->T[8 * k + e] = rows[k][e];
            s += rows[k][e] * rows[k][e];
        }
        m->n[k] = s;
    }
}

void row_angles(const adct_matrix &m, double *out) {
    const DctRows r = dct_rows();
    for (int k = 0; k < 8; ++k) {
        double dot = 0.0;
        for (int e = 0; e < 8; ++e) dot += m.T[8 * k + e] * r.c[8 * k + e];
        const double c = dot / sqrt(double(m.n[k]));
        out[k] = acos(std::max(-1.0, std::min(1.0, c)));
    }
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

adct_status adct_derive_transform(const int8_t *P, int nP, int mode, const uint8_t *orders,
                                  int n_orders, int fix_rows_1_5, adct_matrix *out, int cap_out,
                                  int *n_out, double *angles_out, int64_t *leaves_out,
                                  int64_t *dead_out, adct_stream_t stream) {
    if (mode != ADCT_SEARCH_CLOSURE && mode != ADCT_SEARCH_CANONICAL)
        return fail(ADCT_EINVAL, "mode must be ADCT_SEARCH_CLOSURE or ADCT_SEARCH_CANONICAL");
    if (!n_out) return fail(ADCT_EINVAL, "n_out is null");
    if (cap_out < 0 || (cap_out > 0 && !out)) return fail(ADCT_EINVAL, "out is null");
    std::vector<int> free_rows;
    for (int k = 0; k < 8; ++k)
        if (!fix_rows_1_5 || (k != 0 && k != 4)) free_rows.push_back(k);
    const int nf = int(free_rows.size());
    // the order list: given, or every permutation of the free rows
    std::vector<std::vector<int>> ords;
    if (orders) {
        if (n_orders < 1) return fail(ADCT_ERANGE, "n_orders must be >= 1");
        for (int o = 0; o < n_orders; ++o) {
            std::vector<int> ord(orders + int64_t(o) * nf, orders + int64_t(o + 1) * nf);
            std::vector<int> srt = ord;
            std::sort(srt.begin(), srt.end());
            if (srt != free_rows) return fail(ADCT_EINVAL, "each order must be a permutation of the free rows");
            ords.push_back(ord);
        }
    } else {
        std::vector<int> ord = free_rows;
        do ords.push_back(ord);
        while (std::next_permutation(ord.begin(), ord.end()));
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Space sp;
    adct_status st = build_space(P, nP, sp, s);
    if (st) return st;

    Tree tr;
    tr.add_node();
    for (const auto &ord : ords) {
        int node = 0;
        tr.leaves[0]++;
        for (int k : ord) {
            auto it = tr.kids[node].find(k);
            int nx;
            if (it == tr.kids[node].end()) {
                nx = tr.add_node();
                tr.kids[node][k] = nx;
            } else {
                nx = it->second;
            }
            node = nx;
            tr.leaves[node]++;
        }
    }

    State root;
    memset(&root, 0, sizeof(root));
    root.node = 0;
    const int8_t r0[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    const int8_t r4[8] = {1, -1, -1, 1, 1, -1, -1, 1};
    if (fix_rows_1_5) {
        memcpy(root.rows[0], r0, 8);
        memcpy(root.rows[4], r4, 8);
        root.set[0] = root.set[4] = true;
    }
    // the root's feasible list: every candidate orthogonal to the fixed rows
    int cur_slot = 8, nxt_slot = 9;
    uint32_t *lists_p = nullptr;
    int *dlen_p = nullptr;
    if ((st = cached_n(sp, cur_slot, sp.n, &lists_p))) return st;
    if ((st = cached_n(sp, 11, 1, &dlen_p))) return st;
    ADCT_HIP(hipMemsetAsync(dlen_p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_root_list, dim3(unsigned(std::min<int64_t>((sp.n + 255) / 256, 2048))), dim3(256), 0, s,
                       sp.n, (const uint2 *)sp.vec, pack8(r0), pack8(r4), fix_rows_1_5 ? 2 : 0,
                       lists_p, dlen_p);
    ADCT_HIP(hipGetLastError());
    int root_len = 0;
    ADCT_HIP(hipMemcpyAsync(&root_len, dlen_p, sizeof(int), hipMemcpyDeviceToHost, s));
    ADCT_HIP(hipStreamSynchronize(s));
    root.loff = 0;
    root.llen = root_len;
    std::map<MatKey, adct_matrix> found;
    int64_t leaves = 0, dead = 0;
    std::vector<State> frontier{root};
    while (!frontier.empty()) {
        std::vector<Query> qs;
        std::vector<std::pair<int, int>> qmeta;          // (state, row)
        for (size_t si = 0; si < frontier.size(); ++si) {
            const State &S = frontier[si];
            for (const auto &kv : tr.kids[S.node]) {
                Query q;
                q.off = S.loff;
                q.len = S.llen;
                q.row = kv.first;
                qs.push_back(q);
                qmeta.emplace_back(int(si), kv.first);
            }
        }
        std::vector<std::vector<Cand>> res;
        std::vector<char> isdead;
        if ((st = run_queries(sp, lists_p, qs, res, isdead, s))) return st;
        std::vector<State> next;
        for (size_t q = 0; q < qs.size(); ++q) {
            const State &S = frontier[qmeta[q].first];
            const int row = qmeta[q].second;
            const int child = tr.kids[S.node].at(row);
            if (isdead[q]) {
                dead += tr.leaves[child];
                continue;
            }
            std::vector<Cand> grp = top_group(res[q]);
            if (mode == ADCT_SEARCH_CANONICAL) {
                canonical_sort(grp);
                grp.resize(1);
            }
            for (const Cand &c : grp) {
                State N = S;
                N.node = child;
                decode_index(sp, c.idx, N.rows[row]);
                N.set[row] = true;
                N.chosen = uint32_t(c.idx - 1);
                if (tr.kids[child].empty()) {
                    adct_matrix m;
                    fill_matrix(N.rows, &m);
                    MatKey key;
                    memcpy(key.b.data(), m.T, 64);
                    found[key] = m;
                    leaves++;
                } else {
                    next.push_back(N);
                }
            }
        }
        // the next level's feasible lists: each child filters its parent's list
        if (!next.empty()) {
            std::vector<FilterJob> jobs(next.size());
            int64_t total = 0;
            for (size_t j = 0; j < next.size(); ++j) {
                jobs[j].in_off = next[j].loff;
                jobs[j].in_len = next[j].llen;
                jobs[j].out_off = total;
                jobs[j].chosen = next[j].chosen;
                total += next[j].llen;
            }
            const int nj = int(next.size());
            if (total > (int64_t(1) << 33))
                return fail(ADCT_ERANGE, "the next depth's feasible lists would exceed 32 GB (fix rows 1 and 5, "
                                         "or search fewer orders)");
            uint32_t *nl_p = nullptr;
            FilterJob *dj_p = nullptr;
            int *dl_p = nullptr;
            if ((st = cached_n(sp, nxt_slot, total, &nl_p))) return st;
            if ((st = cached_n(sp, 10, nj, &dj_p))) return st;
            if ((st = cached_n(sp, 11, nj, &dl_p))) return st;
            ADCT_HIP(hipMemcpyAsync(dj_p, jobs.data(), sizeof(FilterJob) * nj, hipMemcpyHostToDevice, s));
            ADCT_HIP(hipMemsetAsync(dl_p, 0, sizeof(int) * nj, s));
            int64_t maxlen = 1;
            for (const FilterJob &j : jobs) maxlen = std::max<int64_t>(maxlen, j.in_len);
            const unsigned chunks = unsigned(std::min<int64_t>((maxlen + 255) / 256, 64));
            for (int y0 = 0; y0 < nj; y0 += 65535) {
                const int ny = std::min(nj - y0, 65535);
                hipLaunchKernelGGL(k_filter, dim3(chunks, ny), dim3(256), 0, s, (const uint2 *)sp.vec,
                                   lists_p, dj_p + y0, nl_p,
                                   dl_p + y0);
                ADCT_HIP(hipGetLastError());
            }
            std::vector<int> lens(nj);
            ADCT_HIP(hipMemcpyAsync(lens.data(), dl_p, sizeof(int) * nj, hipMemcpyDeviceToHost, s));
            ADCT_HIP(hipStreamSynchronize(s));
            for (int j = 0; j < nj; ++j) {
                next[j].loff = jobs[j].out_off;
                next[j].llen = lens[j];
            }
            lists_p = nl_p;               // the parent arena is reused two depths on
            std::swap(cur_slot, nxt_slot);
        }
        frontier.swap(next);
    }
    *n_out = int(found.size());
    if (leaves_out) *leaves_out = leaves;
    if (dead_out) *dead_out = dead;
    int i = 0;
    for (const auto &kv : found) {
        if (i >= cap_out) break;
        out[i] = kv.second;
        if (angles_out) row_angles(kv.second, angles_out + 8 * i);
        ++i;
    }
    if (int(found.size()) > cap_out) return fail(ADCT_ECAP, "output capacity too small");
    return ADCT_OK;
}

adct_status adct_search_topk(const int8_t *P, int nP, int k, int primitive, int8_t *vec_out,
                             int64_t *idx_out, double *cos_out, adct_stream_t stream) {
    if (k < 1) return fail(ADCT_ERANGE, "k must be >= 1");
    if (!vec_out || !idx_out || !cos_out) return fail(ADCT_EINVAL, "outputs are required");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Space sp;
    adct_status st = build_space(P, nP, sp, s);
    if (st) return st;
    DevBuf dhist;
    if ((st = dalloc<unsigned>(dhist, 8 * kHistBins))) return st;
    void *codes = nullptr;
    if ((st = cached(sp, 2, size_t(sp.n) * sizeof(uint2), &codes))) return st;
    ADCT_HIP(hipMemsetAsync(dhist.p, 0, sizeof(unsigned) * 8 * kHistBins, s));
    const unsigned grid = unsigned(std::min<int64_t>((sp.n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_hist, dim3(grid), dim3(256), 0, s, sp.n, (const uint2 *)sp.vec,
                       (const uint8_t *)sp.prim, primitive, (const double *)sp.inv.p, dct_rows(),
                       (unsigned *)dhist.p, (uint2 *)codes);
    ADCT_HIP(hipGetLastError());
    std::vector<unsigned> hist(8 * kHistBins);
    ADCT_HIP(hipMemcpyAsync(hist.data(), dhist.p, sizeof(unsigned) * hist.size(), hipMemcpyDeviceToHost, s));
    ADCT_HIP(hipStreamSynchronize(s));
    // per row the highest bin whose cumulative count (from the smallest angle)
    // reaches k + a margin.  Exact ties share a bin, so they are collected
    // whole; a chain of near-ties (each within kTieEps) could still cross the
    // threshold bin, so after ranking the tie group at position k must end
    // before the last collected candidate.  Rows where it does not lower
    // their threshold by one bin and the rows are collected again.
    Thresholds th;
    int bins[8];
    int64_t cums[8];
    for (int r = 0; r < 8; ++r) {
        int64_t cum = 0;
        int bn = kHistBins - 1;
        for (; bn >= 0; --bn) {
            cum += hist[r * kHistBins + bn];
            if (cum >= int64_t(k) + 64) break;
        }
        if (bn < 0) bn = 0;
        bins[r] = bn;
        cums[r] = cum;
    }
    for (;;) {
        int64_t total = 0;
        for (int r = 0; r < 8; ++r) {
            th.bin[r] = bins[r];
            th.cap[r] = cums[r];
            th.off[r] = total;
            total += cums[r];
        }
        DevBuf didx, dcos, dcnt;
        if ((st = dalloc<int64_t>(didx, total))) return st;
        if ((st = dalloc<double>(dcos, total))) return st;
        if ((st = dalloc<unsigned long long>(dcnt, 8))) return st;
        ADCT_HIP(hipMemsetAsync(dcnt.p, 0, sizeof(unsigned long long) * 8, s));
        bool bytes_ok = true;
        for (int r = 0; r < 8; ++r) bytes_ok &= th.bin[r] <= 254;
        if (bytes_ok)
            hipLaunchKernelGGL(k_topk_collect_codes, dim3(grid), dim3(256), 0, s, sp.n, (const uint2 *)codes,
                               (const uint2 *)sp.vec, (const double *)sp.inv.p, dct_rows(), th,
                               (int64_t *)didx.p, (double *)dcos.p, (unsigned long long *)dcnt.p);
        else
            hipLaunchKernelGGL(k_topk_collect, dim3(grid), dim3(256), 0, s, sp.n, (const uint2 *)sp.vec,
                               (const uint8_t *)sp.prim, primitive, (const double *)sp.inv.p, dct_rows(), th,
                               (int64_t *)didx.p, (double *)dcos.p, (unsigned long long *)dcnt.p);
        ADCT_HIP(hipGetLastError());
        std::vector<int64_t> idx(std::max<int64_t>(total, 1));
        std::vector<double> cs(std::max<int64_t>(total, 1));
        std::vector<unsigned long long> cnt(8);
        ADCT_HIP(hipMemcpyAsync(idx.data(), didx.p, sizeof(int64_t) * total, hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipMemcpyAsync(cs.data(), dcos.p, sizeof(double) * total, hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipMemcpyAsync(cnt.data(), dcnt.p, sizeof(unsigned long long) * 8, hipMemcpyDeviceToHost, s));
        ADCT_HIP(hipStreamSynchronize(s));
        bool again = false;
        for (int r = 0; r < 8; ++r) {
            if (int64_t(cnt[r]) != th.cap[r]) return fail(ADCT_EDEVICE, "top-k collection count mismatch");
            std::vector<Cand> c(size_t(th.cap[r]));
            for (int64_t j = 0; j < th.cap[r]; ++j) {
                c[j].idx = idx[th.off[r] + j] + 1;
                c[j].cos = cs[th.off[r] + j];
                int8_t v[8];
                decode_index(sp, c[j].idx, v);
                c[j].norm2 = norm2_of(v);
            }
            canonical_sort(c);
            if (int64_t(c.size()) < k) return fail(ADCT_ERANGE, "fewer candidates than k");
            size_t e = size_t(k) - 1;
            while (e + 1 < c.size() && c[e].cos - c[e + 1].cos <= kTieEps) ++e;
            if (e + 1 == c.size() && bins[r] > 0) {
                // the group may go on below the threshold: take one more bin
                --bins[r];
                cums[r] += hist[r * kHistBins + bins[r]];
                again = true;
                continue;
            }
            for (int j = 0; j < k; ++j) {
                decode_index(sp, c[j].idx, vec_out + (int64_t(r) * k + j) * 8);
                idx_out[int64_t(r) * k + j] = c[j].idx;
                cos_out[int64_t(r) * k + j] = c[j].cos;
            }
        }
        if (!again) return ADCT_OK;
    }
}

adct_status adct_orthogonal_tuples(const int8_t *lists, const int *len, int32_t *out, int64_t cap,
                                   int64_t *n_total, adct_stream_t stream) {
    if (!lists || !len || !n_total) return fail(ADCT_EINVAL, "lists, len and n_total are required");
    if (cap < 0 || (cap > 0 && !out)) return fail(ADCT_EINVAL, "out is null");
    int kmax = 0, base[8], tot = 0;
    for (int r = 0; r < 8; ++r) {
        if (len[r] < 0) return fail(ADCT_ERANGE, "negative list length");
        base[r] = tot;
        tot += len[r];
        kmax = std::max(kmax, len[r]);
    }
    *n_total = 0;
    for (int r = 0; r < 8; ++r)
        if (len[r] == 0) return ADCT_OK;
    const int words = (kmax + 63) / 64;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::vector<uint2> packed(tot);
    for (int i = 0; i < tot; ++i) packed[i] = pack8(lists + 8 * int64_t(i));
    DevBuf dl, dlen, dbase, dbits;
    adct_status st;
    if ((st = dalloc<uint2>(dl, tot))) return st;
    if ((st = dalloc<int>(dlen, 8))) return st;
    if ((st = dalloc<int>(dbase, 8))) return st;
    const int64_t nbits = int64_t(28) * kmax * words;
    if ((st = dalloc<unsigned long long>(dbits, nbits))) return st;
    ADCT_HIP(hipMemcpyAsync(dl.p, packed.data(), sizeof(uint2) * tot, hipMemcpyHostToDevice, s));
    ADCT_HIP(hipMemcpyAsync(dlen.p, len, sizeof(int) * 8, hipMemcpyHostToDevice, s));
    ADCT_HIP(hipMemcpyAsync(dbase.p, base, sizeof(int) * 8, hipMemcpyHostToDevice, s));
    const int64_t threads = int64_t(kmax) * words;
    hipLaunchKernelGGL(k_ortho_bits, dim3(unsigned((threads + 255) / 256), 28), dim3(256), 0, s,
                       (const uint2 *)dl.p, (const int *)dlen.p, (const int *)dbase.p, kmax, words,
                       (unsigned long long *)dbits.p);
    ADCT_HIP(hipGetLastError());
    std::vector<unsigned long long> bits(nbits);
    ADCT_HIP(hipMemcpyAsync(bits.data(), dbits.p, sizeof(unsigned long long) * nbits, hipMemcpyDeviceToHost, s));
    ADCT_HIP(hipStreamSynchronize(s));
    auto pair_index = [](int r1, int r2) {             // r1 < r2, row-major over the upper triangle
        return r1 * 7 - r1 * (r1 - 1) / 2 + (r2 - r1 - 1);
    };
    // iterative depth-first search; cand[r] = AND of the orthogonality rows of
    // the vectors chosen for rows < r
    std::vector<std::vector<unsigned long long>> cand(8, std::vector<unsigned long long>(words));
    int pos[8];
    int64_t count = 0;
    int r = 0;
    for (int w = 0; w < words; ++w) cand[0][w] = ~0ull;
    pos[0] = -1;
    while (r >= 0) {
        int a = pos[r] + 1;
        while (a < len[r] && !((cand[r][a >> 6] >> (a & 63)) & 1ull)) ++a;
        if (a >= len[r]) {
            --r;
            continue;
        }
        pos[r] = a;
        if (r == 7) {
            if (count < cap)
                for (int q = 0; q < 8; ++q) out[count * 8 + q] = pos[q];
            ++count;
            continue;
        }
        const int nr = r + 1;
        for (int w = 0; w < words; ++w) {
            unsigned long long m = ~0ull;
            for (int q = 0; q <= r; ++q)
                m &= bits[(int64_t(pair_index(q, nr)) * kmax + pos[q]) * words + w];
            cand[nr][w] = m;
        }
        pos[nr] = -1;
        r = nr;
    }
    *n_total = count;
    return ADCT_OK;
}

}  // extern "C"
