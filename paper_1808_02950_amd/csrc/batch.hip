// Batched evaluation: many images of uneven sizes x several transforms x every
// retention level r in one persistent launch (the rate-distortion sweep of
// Sec. 6.1.1, where the paper averages MSE / PSNR over images for each r).
//
// A work item is one tile of 64 blocks of one image and a group of transforms;
// one wave owns an item, one lane owns one block.  Per transform the lane
// computes the forward transform once, stages its coefficients in LDS (zig-zag
// order, lane-interleaved so every read is conflict-free), then walks the
// zig-zag scan: step j adds coefficient j's outer product to the block's
// reconstruction numerator, rounds, clips and scores it, giving the squared
// error for r = j + 1.  Integer transforms accumulate exact integer numerators
// over L = lcm(n)^2 (bit-exact against the oracle); the exact DCT accumulates in
// float64.  Each step's per-lane errors are summed across the wave and added to
// the [image][transform][r] table.
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
    int32_t split;                    // transform groups per tile
    int32_t total_tiles;
    int32_t tids[kMaxBatchTransforms];
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

// Per-wave coefficient staging: 64 coefficients x 64 lanes, entry [z][lane]
// (float64 for the DCT, int32 for integer transforms).  Single-wave
// workgroups, so each wave owns the whole array.
__shared__ double g_stage[64 * 64];

// A[:, Y] += t u for a wave-uniform t in {0, +-1, +-2}
template <int Y>
__device__ __forceinline__ void add_col(int (&A)[8][8], const int (&u)[8], int t) {
    if (t == 1) {
#pragma unroll
        for (int x = 0; x < 8; ++x) A[x][Y] += u[x];
    } else if (t == -1) {
#pragma unroll
        for (int x = 0; x < 8; ++x) A[x][Y] -= u[x];
    } else if (t == 2) {
#pragma unroll
        for (int x = 0; x < 8; ++x) A[x][Y] += u[x] + u[x];
    } else if (t == -2) {
#pragma unroll
        for (int x = 0; x < 8; ++x) A[x][Y] -= u[x] + u[x];
    }
}

template <size_t... Ys>
__device__ __forceinline__ void add_outer(int (&A)[8][8], const int (&u)[8], const int8_t (&row)[8],
                                          std::index_sequence<Ys...>) {
    (add_col<int(Ys)>(A, u, int(row[Ys])), ...);
}

// column pass of the forward for column Lc: Y[:, Lc] = T Z[:, Lc]; stores
// V = Y c_k c_l at the coefficient's zig-zag slot
template <int ID, int Lc>
__device__ __forceinline__ void fwd_col(const int (&Z)[8][8], int *lds, int lane) {
    int in[8], out[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) in[x] = Z[x][Lc];
    fwd_full<ID>(in, out);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        lds[zz_pos(k, Lc) * 64 + lane] = out[k] * (Tf<ID>::c(k) * Tf<ID>::c(Lc));
}

template <int ID, size_t... Ls>
__device__ __forceinline__ void fwd_cols(const int (&Z)[8][8], int *lds, int lane, std::index_sequence<Ls...>) {
    (fwd_col<ID, int(Ls)>(Z, lds, lane), ...);
}

// the same for the float64 DCT: B[:, Lc] = C Z[:, Lc] (even/odd butterfly)
template <int Lc>
__device__ __forceinline__ void dct_col(const double (&Z)[8][8], double *lds, int lane) {
    double se[4], de[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        se[m] = Z[m][Lc] + Z[7 - m][Lc];
        de[m] = Z[m][Lc] - Z[7 - m][Lc];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) acc = fma(kDct.c[8 * k + m], (k & 1) ? de[m] : se[m], acc);
        lds[zz_pos(k, Lc) * 64 + lane] = acc;
    }
}

template <size_t... Ls>
__device__ __forceinline__ void dct_cols(const double (&Z)[8][8], double *lds, int lane, std::index_sequence<Ls...>) {
    (dct_col<int(Ls)>(Z, lds, lane), ...);
}

// round-half-to-even(n / L) clipped to [0, 255], exact
template <int32_t L>
__device__ __forceinline__ int rne_clip(int n) {
    const int nc = min(max(n, 0), 255 * L);
    const uint32_t u = 2u * uint32_t(nc) + uint32_t(L);
    const uint32_t q = u / uint32_t(2 * L);
    const bool tie = (u == uint32_t(__umul24(q, uint32_t(2 * L))));
    return int(q) - int(tie & (q & 1u));
}

// Integer transform: exact incremental reconstruction over the zig-zag scan.
struct Pix {
    uint32_t w[8][2];
};

// One transform's sweep over the zig-zag scan for the lane's block.  A real
// (non-inlined) function per transform, so each gets its own register
// allocation; `out` points at the transform's r_lo..r_hi row of the table.
template <int ID>
__device__ __noinline__ void sweep_int(const Pix P, bool active, unsigned long long *out, int r_lo, int r_hi) {
    const uint32_t (&pix)[8][2] = P.w;
    int *lds = reinterpret_cast<int *>(g_stage);
    constexpr int32_t L = Tf<ID>::L();
    const int lane = threadIdx.x & 63;
    // forward Y = T A T^T; V_z = Y(k, l) c_k c_l at zig-zag position z -> LDS
    int Z[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        int in[8], out[8];
#pragma unroll
        for (int y = 0; y < 8; ++y) in[y] = pix_at(pix, x, y);
        fwd_full<ID>(in, out);
#pragma unroll
        for (int l = 0; l < 8; ++l) Z[x][l] = out[l];
    }
    fwd_cols<ID>(Z, lds, lane, std::make_index_sequence<8>{});
    __builtin_amdgcn_wave_barrier();
    int A[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) A[x][y] = 0;
    const uint32_t e_pix = pix_energy(pix);
    for (int j = 0; j < r_hi; ++j) {
        const int v = lds[j * 64 + lane];
        const int k = kZZDev.k[j], l = kZZDev.l[j];           // wave-uniform
        const Mat8 &T = kMatDev[ID];
        int u[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) u[x] = v * int(T.m[k][x]);
        // A += u t_l^T; t_l entries are 0, +-1, +-2 and wave-uniform
        add_outer(A, u, T.m[l], std::make_index_sequence<8>{});
        uint32_t sq = e_pix, cross = 0;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int q[8];
#pragma unroll
            for (int y = 0; y < 8; ++y) q[y] = rne_clip<L>(A[x][y]);
            score_row(q, pix[x][0], pix[x][1], sq, cross);
        }
        unsigned err = sq - 2u * cross;
        if (j + 1 >= r_lo) {
            err = wave_add(active ? err : 0u);
            if (lane == 0 && err) atomicAdd(out + (j + 1 - r_lo), (unsigned long long)err);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Exact DCT: float64 incremental reconstruction over the zig-zag scan.
__device__ __noinline__ void sweep_dct(const Pix P, bool active, unsigned long long *out, int r_lo, int r_hi) {
    const uint32_t (&pix)[8][2] = P.w;
    double *lds = g_stage;
    const int lane = threadIdx.x & 63;
    {
        // row pass Z = A C^T with the even/odd butterfly (exact integer sums first)
        double Z[8][8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int sm[4], dm[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sm[m] = pix_at(pix, x, m) + pix_at(pix, x, 7 - m);
                dm[m] = pix_at(pix, x, m) - pix_at(pix, x, 7 - m);
            }
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < 4; ++m) acc = fma(double((l & 1) ? dm[m] : sm[m]), kDct.c[8 * l + m], acc);
                Z[x][l] = acc;
            }
        }
        // column pass B = C Z, written to LDS in zig-zag order
        dct_cols(Z, lds, lane, std::make_index_sequence<8>{});
    }
    __builtin_amdgcn_wave_barrier();
    // two passes over half-blocks of 4 rows keep 32 float64 accumulators live
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
        for (int j = 0; j < r_hi; ++j) {
            const double b = lds[j * 64 + lane];
            const int k = kZZDev.k[j], l = kZZDev.l[j];         // wave-uniform
            double u[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) u[x] = b * kDct.c[8 * k + 4 * h + x];
#pragma unroll
            for (int y = 0; y < 8; ++y) {
                const double cl = kDct.c[8 * l + y];
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
    __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_batch(const BatchArgs a) {
    const int lane = threadIdx.x;
    const int items = a.total_tiles * a.split;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tile = it / a.split, grp = it - tile * a.split;
        int i = 0;                                              // image of this tile (uniform)
        int lo = 0, hi = a.n_images - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.img[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
        }
        i = lo;
        const BatchImg &I = a.img[i];
        const int b = (tile - I.tile_start) * 64 + lane;
        const bool active = b < I.nblocks;
        const int bb = active ? b : 0;
        const int by = bb / I.nbx, bx = bb - by * I.nbx;
        const uint8_t *src = a.base + I.offset + int64_t(8 * by) * I.pitch + 8 * bx;
        Pix P;
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            const u32x2 v = *(const u32x2 *)(src + int64_t(x) * I.pitch);
            P.w[x][0] = v.x;
            P.w[x][1] = v.y;
        }
        const int nr = a.r_hi - a.r_lo + 1;
        for (int ti = grp; ti < a.n_transforms; ti += a.split) {
            unsigned long long *out = a.sse + (int64_t(i) * a.n_transforms + ti) * nr;
            switch (a.tids[ti]) {
                case ADCT_DCT: sweep_dct(P, active, out, a.r_lo, a.r_hi); break;
                case ADCT_T1: sweep_int<ADCT_T1>(P, active, out, a.r_lo, a.r_hi); break;
                case ADCT_T2: sweep_int<ADCT_T2>(P, active, out, a.r_lo, a.r_hi); break;
                case ADCT_LO: sweep_int<ADCT_LO>(P, active, out, a.r_lo, a.r_hi); break;
                case ADCT_T6: sweep_int<ADCT_T6>(P, active, out, a.r_lo, a.r_hi); break;
                case ADCT_RDCT: sweep_int<ADCT_RDCT>(P, active, out, a.r_lo, a.r_hi); break;
                default: sweep_int<ADCT_T4>(P, active, out, a.r_lo, a.r_hi); break;
            }
        }
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

adct_status enqueue(const BatchArgs &a, int wgs_per_cu, hipStream_t s) {
    const int64_t n = int64_t(a.n_images) * a.n_transforms * (a.r_hi - a.r_lo + 1);
    hipLaunchKernelGGL(k_zero, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a.sse, n);
    ADCT_HIP(hipGetLastError());
    const int cus = device_cus();
    if (cus <= 0) return fail(ADCT_EDEVICE, "cannot query the device");
    const int64_t items = int64_t(a.total_tiles) * a.split;
    const int grid = int(std::max<int64_t>(1, std::min<int64_t>(items, int64_t(wgs_per_cu) * cus)));
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(64), 0, s, a);
    ADCT_HIP(hipGetLastError());
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
    a.split = split;
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
        for (int split = 1; split <= p->args.n_transforms; ++split) {
            if (p->args.n_transforms % split) continue;
            for (int w : {2, 3, 4, 5, 6, 8}) {
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
