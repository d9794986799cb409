// Structural similarity (SSIM) of a reconstruction against its original, the
// third figure of merit of Sec. 6.1.1, with the definition of the reference it
// cites: local weighted statistics over an 11 x 11 Gaussian window (sigma 1.5,
// unit sum) at every position where the window fits, C1 = (0.01 * 255)^2,
// C2 = (0.03 * 255)^2, and the mean of the map per plane.
//
// One wave computes a tile of the map: 64 output columns (one per lane) x 176
// output rows.  Input rows stream through it once: each row's two pixels per
// position (loaded one row ahead) go to a per-wave LDS row (x | y << 16),
// every lane sums its 11
// horizontal neighbours' x, y, x^2, y^2, xy with the 1-D weights (mirrored taps
// added as exact integers first, the weights being symmetric), and that row
// of horizontal sums is folded into the 11 output rows it reaches with the
// vertical weights.  Eleven rotating accumulators hold those rows; with the row
// loop unrolled by 11 every accumulator index is a compile-time constant.  An
// accumulator is complete when its last input row arrives: the lane then
// evaluates SSIM there.  Pixels are centred at 128 before the products (the
// variances and covariance do not change) and everything accumulates in
// float64.  Each plane's map sum is accumulated as a 2^-36 fixed-point 64-bit
// integer, so the per-plane result does not depend on the order of the tiles.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "adct_internal.hpp"
#include "xcd.hpp"

namespace adct {
namespace {

constexpr int kWin = 11;
constexpr int kTileRows = 176;                // output rows per tile (a multiple of 11)
constexpr double kC1 = 6.5025;                // (0.01 * 255)^2
constexpr double kC2 = 58.5225;               // (0.03 * 255)^2
constexpr double kFix = 68719476736.0;        // 2^36

struct SsimPlane {
    int64_t off;
    int32_t pitch, H, W;
    int32_t strips, tile_start;               // 64-column strips; first tile of the plane in a frame
};

struct SsimArgs {
    const uint8_t *ref;
    const uint8_t *test;
    int64_t fs_ref, fs_test;
    unsigned long long *acc;                  // [frame][plane] fixed-point map sums, then means
    int32_t n_frames, n_planes, tiles_per_frame, pad;
    SsimPlane pl[kMaxPlanes];
    double w[kWin];                           // 1-D Gaussian weights, unit sum
};

// SSIM at one position from the window's sums of x, y, x^2, y^2, xy (pixels
// centred at 128)
__device__ __forceinline__ double ssim_at(const double (&s)[5]) {
    const double mx = s[0], my = s[1];
    const double vx = s[2] - mx * mx, vy = s[3] - my * my, cxy = s[4] - mx * my;
    const double ux = mx + 128.0, uy = my + 128.0;
    return ((2.0 * ux * uy + kC1) * (2.0 * cxy + kC2)) / ((ux * ux + uy * uy + kC1) * (vx + vy + kC2));
}

// one input row (relative index i = i0 + U) of the tile; U is the row's
// position in its group of 11, so every accumulator slot is a constant
// the four pixel bytes a lane loads for one input row (its column and, for
// lanes 0..9, the column 64 further), issued one row ahead of their use
struct RowPix {
    uint32_t ra, ta, rb, tb;
};

__device__ __forceinline__ void load_row(const uint8_t *rb, const uint8_t *tb, const SsimPlane &P, int r, int ca,
                                         int cb, int lane, RowPix &v) {
    const int64_t base = int64_t(std::min(r, P.H - 1)) * P.pitch;
    v.ra = rb[base + ca];
    v.ta = tb[base + ca];
    if (lane < kWin - 1) {
        v.rb = rb[base + cb];
        v.tb = tb[base + cb];
    }
}

template <int U>
__device__ __forceinline__ void ssim_row(const SsimArgs &a, const uint8_t *rb, const uint8_t *tb, const SsimPlane &P,
                                         int r0, int i0, int nout, int ca, int cb, int lane, uint32_t *row,
                                         RowPix &nx, double (&acc)[kWin][5], double &sum, bool col_ok) {
    const int i = i0 + U;
    if (i >= nout + kWin - 1) return;                          // wave-uniform
    const RowPix cur = nx;
    if (i + 1 < nout + kWin - 1) load_row(rb, tb, P, r0 + i + 1, ca, cb, lane, nx);
    row[lane] = cur.ra | (cur.ta << 16);
    if (lane < kWin - 1) row[64 + lane] = cur.rb | (cur.tb << 16);
    __builtin_amdgcn_wave_barrier();
    int x[kWin], y[kWin];
#pragma unroll
    for (int b = 0; b < kWin; ++b) {
        const uint32_t v = row[lane + b];
        x[b] = int(v & 0xffffu) - 128;
        y[b] = int(v >> 16) - 128;
    }
    __builtin_amdgcn_wave_barrier();
    // the weights are symmetric: taps b and 10 - b are added as exact integers first
    const double w5 = a.w[5];
    double h[5] = {w5 * double(x[5]), w5 * double(y[5]), w5 * double(x[5] * x[5]), w5 * double(y[5] * y[5]),
                   w5 * double(x[5] * y[5])};
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const int c = kWin - 1 - b;
        const double wb = a.w[b];
        h[0] = fma(wb, double(x[b] + x[c]), h[0]);
        h[1] = fma(wb, double(y[b] + y[c]), h[1]);
        h[2] = fma(wb, double(x[b] * x[b] + x[c] * x[c]), h[2]);
        h[3] = fma(wb, double(y[b] * y[b] + y[c] * y[c]), h[3]);
        h[4] = fma(wb, double(x[b] * y[b] + x[c] * y[c]), h[4]);
    }
    // this row feeds output rows o = i - d, d = 0..10, of slot (U - d) mod 11 =
    // o mod 11; it is the first row of output o = i (d = 0), which starts the
    // slot afresh, so a completed slot needs no clearing
#pragma unroll
    for (int d = 0; d < kWin; ++d) {
        if (d <= i && i - d < nout) {
            double(&s)[5] = acc[(U - d + kWin) % kWin];
            const double wd = a.w[d];
#pragma unroll
            for (int q = 0; q < 5; ++q) s[q] = d == 0 ? wd * h[q] : fma(wd, h[q], s[q]);
        }
    }
    // output row o = i - 10 is complete
    if (i >= kWin - 1 && i - (kWin - 1) < nout) {
        const double(&s)[5] = acc[(U + 1) % kWin];
        if (col_ok) sum += ssim_at(s);
    }
}

// Workgroups are renumbered so that each XCD takes one contiguous run of
// tiles: horizontally adjacent strips, which share the 128-byte lines at their
// seams, then run on the same L2 at about the same time.
__global__ __launch_bounds__(256) void k_ssim(const SsimArgs a) {
    __shared__ uint32_t rows[4][64 + kWin - 1];
    // the wave index read from the first lane, so that the tile, its plane and
    // every row bound below are known to be wave-uniform and the per-row
    // window tests run on the scalar unit instead of as lane masks
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), lane = int(threadIdx.x & 63);
    const int gw = xcd_swizzle(int(blockIdx.x), int(gridDim.x)) * 4 + wave;
    if (gw >= a.n_frames * a.tiles_per_frame) return;          // whole wave leaves
    const int f = gw / a.tiles_per_frame;
    int t = gw - f * a.tiles_per_frame;
    int p = 0;
    while (p + 1 < a.n_planes && t >= a.pl[p + 1].tile_start) ++p;
    const SsimPlane &P = a.pl[p];
    t -= P.tile_start;
    const int band = t / P.strips, strip = t - band * P.strips;
    const int OH = P.H - (kWin - 1), OW = P.W - (kWin - 1);
    const int c0 = strip * 64, r0 = band * kTileRows;
    const int nout = std::min(kTileRows, OH - r0);
    const bool col_ok = c0 + lane < OW;
    // input columns of this lane (and, for lanes 0..9, of the 10 columns past
    // the strip), clamped into the plane: a clamped column only feeds outputs
    // outside the map
    const int ca = std::min(c0 + lane, P.W - 1), cb = std::min(c0 + 64 + lane, P.W - 1);
    const uint8_t *rb = a.ref + int64_t(f) * a.fs_ref + P.off;
    const uint8_t *tb = a.test + int64_t(f) * a.fs_test + P.off;
    uint32_t *row = rows[wave];
    double acc[kWin][5];
#pragma unroll
    for (int k = 0; k < kWin; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[k][q] = 0.0;
    double sum = 0.0;
    RowPix nx = {0u, 0u, 0u, 0u};
    load_row(rb, tb, P, r0, ca, cb, lane, nx);
    for (int i0 = 0; i0 < nout + kWin - 1; i0 += kWin) {
        ssim_row<0>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<1>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<2>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<3>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<4>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<5>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<6>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<7>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<8>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<9>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
        ssim_row<10>(a, rb, tb, P, r0, i0, nout, ca, cb, lane, row, nx, acc, sum, col_ok);
    }
    // fixed point (|map| <= 1, at most 176 entries per lane: below 2^44), then the wave sum
    long long v = llrint(sum * kFix);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) atomicAdd(a.acc + int64_t(f) * a.n_planes + p, (unsigned long long)v);
}

__global__ void k_ssim_zero(unsigned long long *acc, int n) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) acc[i] = 0ull;
}

// fixed-point map sums -> mean SSIM per (frame, plane), in place
__global__ void k_ssim_final(unsigned long long *acc, int n_frames, int n_planes, SsimArgs a) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_frames * n_planes) return;
    const SsimPlane &P = a.pl[i % n_planes];
    const double count = double(P.H - (kWin - 1)) * double(P.W - (kWin - 1));
    const double mean = double((long long)acc[i]) / kFix / count;
    acc[i] = (unsigned long long)__double_as_longlong(mean);
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" adct_status adct_ssim(const uint8_t *ref, int64_t frame_stride_ref, const uint8_t *test,
                                 int64_t frame_stride_test, int n_frames, const adct_plane *planes,
                                 int n_planes, double *ssim_out, adct_stream_t stream) {
    if (!ref || !test || !planes || !ssim_out) return fail(ADCT_EINVAL, "ref, test, planes and ssim_out are required");
    if (n_frames < 1) return fail(ADCT_ERANGE, "n_frames must be >= 1");
    if (n_planes < 1 || n_planes > kMaxPlanes) return fail(ADCT_ERANGE, "n_planes must be in [1, 4]");
    if (reinterpret_cast<uintptr_t>(ssim_out) & 7) return fail(ADCT_EDIM, "ssim_out must be 8-byte aligned");
    if (n_frames > 1 && (frame_stride_ref <= 0 || frame_stride_test <= 0))
        return fail(ADCT_EDIM, "frame strides must be positive for several frames");
    SsimArgs a;
    memset(&a, 0, sizeof(a));
    a.ref = ref;
    a.test = test;
    a.fs_ref = frame_stride_ref;
    a.fs_test = frame_stride_test;
    a.acc = reinterpret_cast<unsigned long long *>(ssim_out);
    a.n_frames = n_frames;
    a.n_planes = n_planes;
    int64_t tiles = 0;
    for (int p = 0; p < n_planes; ++p) {
        const adct_plane &q = planes[p];
        if (q.H < kWin || q.W < kWin || q.pitch < q.W || q.offset < 0)
            return fail(ADCT_EDIM, "each plane needs H, W >= 11, pitch >= W and offset >= 0");
        if (int64_t(q.H) * q.W > (int64_t(1) << 26))
            return fail(ADCT_ERANGE, "planes are limited to 2^26 pixels (fixed-point sum range)");
        SsimPlane &d = a.pl[p];
        d.off = q.offset;
        d.pitch = q.pitch;
        d.H = q.H;
        d.W = q.W;
        d.strips = (q.W - (kWin - 1) + 63) / 64;
        d.tile_start = int32_t(tiles);
        tiles += int64_t(d.strips) * ((q.H - (kWin - 1) + kTileRows - 1) / kTileRows);
    }
    if (tiles * n_frames > (int64_t(1) << 30)) return fail(ADCT_ERANGE, "too many tiles in one call");
    a.tiles_per_frame = int32_t(tiles);
    // 1-D weights: exp(-d^2 / (2 sigma^2)), d = -5..5, normalised (the 2-D window
    // of unit sum is their outer product)
    double s = 0.0;
    for (int d = 0; d < kWin; ++d) s += (a.w[d] = exp(-double((d - 5) * (d - 5)) / (2.0 * 1.5 * 1.5)));
    for (int d = 0; d < kWin; ++d) a.w[d] /= s;
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const int n = n_frames * n_planes;
    hipLaunchKernelGGL(k_ssim_zero, dim3((n + 255) / 256), dim3(256), 0, hs, a.acc, n);
    ADCT_HIP(hipGetLastError());
    const int64_t waves = tiles * n_frames;
    hipLaunchKernelGGL(k_ssim, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, hs, a);
    ADCT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ssim_final, dim3((n + 255) / 256), dim3(256), 0, hs, a.acc, n_frames, n_planes, a);
    ADCT_HIP(hipGetLastError());
    return ADCT_OK;
}
