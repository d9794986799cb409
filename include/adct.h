/* adct.h -- C ABI of the MI355X (gfx950) library for blockwise 8x8 transform
 * coding with low-complexity DCT approximations found by angle similarity
 * (Oliveira, Cintra et al., "Low-complexity 8-point DCT approximation based on
 * angle similarity for image and video coding").
 *
 * Conventions shared by every entry point
 *   - Buffers are owned by the caller.  "device" pointers must point to memory
 *     the current HIP device can access (hipMalloc or torch CUDA tensors);
 *     "host" pointers to ordinary host memory.  The library never frees or
 *     keeps a caller buffer past the call (device work it enqueues reads and
 *     writes them until the stream reaches it).
 *   - `stream` may be 0 (the null stream).  Device work is enqueued on it and
 *     the call returns without waiting, EXCEPT where an entry point says it
 *     synchronises (those that return host results computed on the device).
 *   - Images are 8-bit, row-major, H rows of W pixels, `pitch` bytes between
 *     row starts (pitch >= W).  H and W are multiples of 8.  8x8 blocks are
 *     numbered in raster order: block b = (y/8) * (W/8) + (x/8).
 *   - Coefficients of a block are stored in JPEG zig-zag order (row index =
 *     vertical frequency), the first r of them, so a coefficient array is
 *     [n_blocks][r], n_blocks = (H/8) (W/8).
 *   - Every call returns an adct_status; on error nothing is enqueued and
 *     adct_last_error() returns a message for the calling thread.  No C++
 *     exception crosses this boundary.
 */
#ifndef ADCT_H
#define ADCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *adct_stream_t; /* the same handle as hipStream_t */

typedef enum {
    ADCT_OK = 0,
    ADCT_EINVAL = -1,    /* null pointer where one is required, unknown enum value,
                            custom matrix whose rows are not orthogonal */
    ADCT_EDIM = -2,      /* H or W <= 0 or not a multiple of 8, pitch < W, buffers
                            not aligned as the entry point requires */
    ADCT_ERANGE = -3,    /* r outside [1, 64], quant_step < 0, k < 1, |P| outside [1, 9] ... */
    ADCT_EOVERFLOW = -4, /* the transform's integer stage does not fit the kernel's
                            word size for this mode */
    ADCT_ECAP = -5,      /* output capacity too small; counts still report the need */
    ADCT_EDEVICE = -6,   /* a HIP runtime call failed (message has the HIP error) */
    ADCT_ENOTSUP = -7    /* combination of arguments the library does not implement */
} adct_status;

/* Transforms.  ADCT_DCT is the exact (orthonormal) DCT, a real matrix; the
 * others are integer matrices T whose approximation is C_hat = S T with
 * S = diag(1/sqrt(diag(T T^T))) (Eq. (1)-(2) of the paper; S is the row
 * normalisation, which is what Eq. (2) gives for T with orthogonal rows).
 *   T1, T2  the matrices the paper derives (Sec. 4.1); T1 is the proposed one
 *   LO      Lengwehasatit-Ortega, stored doubled (2 T_LO) so it is integral
 *   T6, T4  Cintra et al. 2014;  RDCT  rounded DCT  (Sec. 2, matrix table)
 *   CUSTOM  a caller's int8 matrix with orthogonal rows, passed in `custom`
 *           (e.g. one adct_derive_transform returned: derive T by Eq. (6),
 *           then code with it, Sec. 3.5 and 6.1.1).  custom->n[k] must equal
 *           (T T^T)_kk > 0 and T T^T must be diagonal, else ADCT_EINVAL.  It
 *           runs kernels that read T at run time: the same results as a
 *           built-in kernel for the same matrix, bit for bit.  Word limits:
 *           lcm(n) <= 2^26 and every partial sum of the exact inverse below
 *           2^61 (ADCT_EOVERFLOW); with a quantiser |Y| < 2^24 (ADCT_ERANGE).
 * Every codec entry point ignores `custom` unless t == ADCT_CUSTOM. */
typedef enum {
    ADCT_DCT = 0,
    ADCT_T1 = 1,
    ADCT_T2 = 2,
    ADCT_LO = 3,
    ADCT_T6 = 4,
    ADCT_RDCT = 5,
    ADCT_T4 = 6,
    ADCT_CUSTOM = 7
} adct_transform_id;

/* A low-complexity matrix: T row-major (T[k*8 + n], row k approximates DCT
 * row k) and n[k] = (T T^T)_kk. */
typedef struct {
    int8_t T[64];
    int32_t n[8];
} adct_matrix;

/* One plane (or image) inside a frame buffer: `offset` bytes from the frame
 * start, H x W pixels, `pitch` bytes per row. */
typedef struct {
    int64_t offset;
    int32_t H, W, pitch;
    int32_t reserved;
} adct_plane;

/* ---------------------------------------------------------------- basics */

/* Message describing the last error on the calling thread ("" if none). */
const char *adct_last_error(void);

/* ABI version of this header (major * 100 + minor). */
int adct_version(void);

/* Launch schedule of the codec kernels (process-wide): the number of resident
 * 4-wave workgroups per compute unit of the persistent grid.  0 (default) =
 * as many as occupancy allows; -1 = no persistence (one 64-block tile per
 * wave); k > 0 = at most k.  Results do not depend on it. */
adct_status adct_codec_set_schedule(int workgroups_per_cu);

/* Device memory the library keeps between calls on the current device, and
 * how to give it back.  The searches (adct_derive_transform and the other
 * search entry points) keep grow-only buffers per device: the enumerated space
 * (8 bytes a vector, 9^8 = 43 M vectors: 344 MB), its flags and bin bytes, the
 * query buffers and the feasible-list arenas (the largest closure searches
 * reach several GB; a search refuses to grow them past 32 GB).
 * adct_coding_gain_sweep keeps one staging buffer (8 (65 n_t + n_rho) bytes
 * at its largest call).  Both are reused by later calls and otherwise kept
 * until the process ends.  This call frees them for the current device (it
 * waits for a search or sweep running on it) and reports the bytes freed
 * (nullable); the next call allocates again.  Batch plans, filter workspaces
 * and the no-allocation sweep's fixed array are not affected. */
adct_status adct_release_caches(int64_t *bytes_released);

/* Fill *out with a built-in matrix (not ADCT_DCT / ADCT_CUSTOM).  Host only. */
adct_status adct_matrix_get(adct_transform_id id, adct_matrix *out);

/* Bound on |T A T^T| over 8-bit blocks A and on the exact inverse numerator
 * for transform `id` (custom: `custom`), retained count r and quantiser step:
 * *fwd_bound, *inv_bound (host, nullable).  Host only; used to pick word
 * sizes and to report ADCT_EOVERFLOW. */
adct_status adct_transform_bounds(adct_transform_id id, const adct_matrix *custom, int r,
                                  int quant_step, int64_t *fwd_bound, int64_t *inv_bound);

/* Host-only validation: the status the codec entry points would return for
 * this transform, retained count r and quantiser step (want_int16: whether
 * int16 coefficients are requested).
 *
 * Quantiser steps and exact halves (Sec. 6.1.1 reconstruction, rounded half
 * to even).  When for every class n_k n_l = mu^2 step / mu has an odd reduced
 * denominator (a multiple of 8 for T1, T2, T6, RDCT, T4, of 32 for LO) no
 * reconstruction can sit exactly on a half and the built-in kernels round in
 * float64.  Any other step in [1, 65535] goes to the run-time-matrix kernels,
 * which decide every pixel within their float64 error bound of a half by the
 * exact sign of its distance in the field generated by the square roots of
 * the row norms (sqrt 10 for T1 and T2, sqrt 3 for T4, sqrt 6 and sqrt 10 for
 * T6, sqrt 2 and sqrt 3 for RDCT, sqrt 3 and sqrt 10 for LO).  ADCT_ENOTSUP if
 * the norms of a custom matrix bring in more than two independent square
 * roots (or p q > 1024); ADCT_ERANGE if the step is too large for the 52-bit
 * components of that decision.  Such steps run at the run-time kernels' speed
 * (one tile per wave, no persistent grid). */
adct_status adct_check_codec_args(adct_transform_id t, const adct_matrix *custom, int r,
                                  int quant_step, int want_int16);

/* ----------------------------------------------------------------- codec */

/* Forward transform of every 8x8 block of `img` (device), keeping the first r
 * zig-zag coefficients (Sec. 6.1.1: B = C_hat A C_hat^T, r retained).
 *   coef_int    device int16 [n_blocks][r], nullable: the exact integer stage
 *               Y = T A T^T (quant_step == 0) or the quantised level
 *               q = round-half-away(B / quant_step) (quant_step > 0), where
 *               B = s_k s_l Y.  Integer transforms only.
 *   coef_scaled device float [n_blocks][r], nullable: B in float32.
 * At least one output must be non-null.  For ADCT_DCT only coef_scaled (and,
 * with quant_step > 0, coef_int holding q) are defined.
 * ADCT_EOVERFLOW if the transform's Y does not fit int16 (LO: use coef_scaled). */
adct_status adct_encode_blocks(const uint8_t *img, int H, int W, int pitch,
                               adct_transform_id t, const adct_matrix *custom,
                               int r, int quant_step,
                               int16_t *coef_int, float *coef_scaled,
                               adct_stream_t stream);

/* Inverse of adct_encode_blocks (Sec. 6.1.1: A = C_hat^T B' C_hat, valid for
 * T with orthogonal rows).  Exactly one input must be non-null:
 *   coef_int    device int16 [n_blocks][r]: Y (quant_step == 0) or q as
 *               written by encode (integer transforms; for ADCT_DCT the
 *               quantised levels, quant_step > 0);
 *   coef_scaled device float32 [n_blocks][r]: B itself, any transform, with
 *               quant_step == 0 (ADCT_EINVAL otherwise); the inverse runs in
 *               float64 (float32 for the exact DCT's matrix cores).
 * Output: `out` (device) H x W uint8 with pitch_out, the reconstruction
 * rounded half-to-even and clipped to [0, 255].  For integer transforms with
 * coef_int and quant_step == 0 the reconstruction is exact (integer
 * arithmetic on the rational result).  Coefficients that no 8-bit block
 * produces may overflow the word sizes the bounds were checked for; the
 * result for them is unspecified (no memory outside the buffers is touched). */
adct_status adct_decode_blocks(const int16_t *coef_int, const float *coef_scaled,
                               int H, int W, uint8_t *out, int pitch_out,
                               adct_transform_id t, const adct_matrix *custom,
                               int r, int quant_step, adct_stream_t stream);

/* Fused encode + decode + error of one image (Sec. 6.1.1, MSE and PSNR).
 *   coef_int   device int16 [n_blocks][r], nullable (as in encode)
 *   recon      device uint8, pitch_out, nullable
 *   sse_dev    device uint64[1], required: set to sum (rec - img)^2
 *   mse_host, psnr_host  host doubles, nullable; if either is non-null the
 *              call synchronises `stream` and fills them (PSNR = +inf when
 *              the error is 0; PSNR = 10 log10(255^2 / MSE)). */
adct_status adct_evaluate_coding(const uint8_t *img, int H, int W, int pitch,
                                 adct_transform_id t, const adct_matrix *custom,
                                 int r, int quant_step,
                                 int16_t *coef_int, uint8_t *recon, int pitch_out,
                                 uint64_t *sse_dev, double *mse_host, double *psnr_host,
                                 adct_stream_t stream);

/* Structural similarity of `test` against `ref` (Sec. 6.1.1 names SSIM as its
 * third figure of merit and cites its definition): for every plane of every
 * frame, the mean over all positions where an 11 x 11 Gaussian window
 * (sigma 1.5, unit sum) fits inside the plane of
 *   ((2 mu_r mu_t + C1)(2 s_rt + C2)) / ((mu_r^2 + mu_t^2 + C1)(s_r^2 + s_t^2 + C2)),
 * C1 = (0.01 * 255)^2, C2 = (0.03 * 255)^2, with the window-weighted means,
 * variances and covariance; no padding, no downsampling.  Frame f of each
 * buffer starts at ref + f * frame_stride_ref (resp. test + f *
 * frame_stride_test), device memory; planes[p] (host array, n_planes <= 4)
 * gives offset, H, W and pitch, the same for both buffers.  ssim_out: device
 * float64 [n_frames][n_planes], 8-byte aligned, overwritten.  Float64
 * arithmetic; each plane's result does not depend on the launch order.
 * Errors: ADCT_EINVAL null pointer; ADCT_ERANGE n_frames < 1, n_planes not in
 * [1, 4], a plane above 2^26 pixels; ADCT_EDIM a plane smaller than 11 x 11,
 * pitch < W, negative offset, unaligned ssim_out, non-positive frame stride
 * with several frames. */
adct_status adct_ssim(const uint8_t *ref, int64_t frame_stride_ref, const uint8_t *test,
                      int64_t frame_stride_test, int n_frames, const adct_plane *planes, int n_planes,
                      double *ssim_out, adct_stream_t stream);

/* Fused encode + decode + error over a stream of frames in ONE launch.
 * Frame f starts at frames + f * frame_stride (device); plane p of it is
 * planes[p] (host array, n_planes <= 4).  Coefficients go to
 * coef + ((f * blocks_per_frame) + plane_block_offset[p] + b) * r, where
 * planes' blocks are numbered consecutively in plane order; recon uses the
 * same offsets and pitches as the input, at recon + f * frame_stride_out.
 * sse (device uint64 [n_frames][n_planes]) is zeroed by the call, then
 * accumulated.  coef and recon are nullable. */
adct_status adct_evaluate_stream(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                 const adct_plane *planes, int n_planes,
                                 adct_transform_id t, const adct_matrix *custom,
                                 int r, int quant_step,
                                 int16_t *coef, uint8_t *recon, int64_t frame_stride_out,
                                 uint64_t *sse, adct_stream_t stream);

/* Measurement helper, not a step of the method: the loads and stores of
 * adct_evaluate_stream for the same arguments (every block read once, the
 * first r int16 coefficients and the reconstruction written, with the same
 * tiles, access widths and persistent grid) and none of its arithmetic: recon
 * receives the input pixels and coef receives bytes of them.  Its duration is
 * the achievable HBM rate of the codec's read / write mix on this device, the
 * ceiling the codec's own rate is compared with.  coef and recon are nullable;
 * errors as for adct_evaluate_stream. */
adct_status adct_stream_bandwidth_probe(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                        const adct_plane *planes, int n_planes, int r, int16_t *coef,
                                        uint8_t *recon, int64_t frame_stride_out, adct_stream_t stream);

/* ---------------------------------------------------------------- 16 / 32 points */

/* The N-point matrix (N = 16 or 32) that the Jridi-Alfalou-Meher construction
 * grows from an 8-point one (Sec. 6.2): row 2i = [t_i, rev(t_i)], row 2i + 1 =
 * [t_i, -rev(t_i)] with t_i row i of the N/2-point matrix (the sign convention
 * of the 16- and 32-point matrices the paper prints; the recursion as written
 * negates some odd rows, which changes no reconstruction).  Only base = ADCT_T1.
 * T: host int8 [N * N] row-major; n: host int32 [N], n[k] = (T T^T)_kk.  Host
 * only.  Errors: ADCT_EINVAL null; ADCT_ENOTSUP other base; ADCT_ERANGE N. */
adct_status adct_jam_matrix(adct_transform_id base, int N, int8_t *T, int32_t *n);

/* Transform coding with N x N blocks and the matrix of adct_jam_matrix (Sec. 6.2
 * for the matrices, Sec. 6.1.1 for the coder): per block B = C_hat A C_hat^T,
 * C_hat = S T, keep the first r coefficients of the N x N JPEG zig-zag scan,
 * optionally quantise (q = round-half-away(B / quant_step)), reconstruct
 * C_hat^T B' C_hat, round half to even, clip to [0, 255] and accumulate the
 * squared error.  Planes of any size: a plane whose sides are not multiples of
 * N is extended by repeating its last row and column, and only its own pixels
 * are written and scored.  frames / planes / recon / frame strides as in
 * adct_evaluate_stream (device memory; recon uses the input's offsets and
 * pitches).  coef (nullable): device int32, 4-byte aligned, [block][r] with
 * the planes' blocks numbered consecutively per frame in plane order, raster
 * order inside a plane; values are the exact integer stage Y (quant_step = 0)
 * or the levels q.  sse: device uint64 [n_frames][n_planes], 8-byte aligned,
 * zeroed by the call then accumulated.  quant_step = 0 reconstructs in exact
 * rational arithmetic; otherwise float64, and quant_step must be a multiple of
 * N (then no reconstruction can sit exactly on a half).
 * Errors: ADCT_EINVAL null frames / planes / sse; ADCT_ENOTSUP base other than
 * ADCT_T1, quant_step not a multiple of N; ADCT_ERANGE N not 16 or 32, r not in
 * [1, N * N], quant_step not in [0, 4096], n_frames < 1, n_planes not in [1, 4],
 * a plane with H or pitch >= 2^24 or H * pitch >= 2^31, too many blocks;
 * ADCT_EDIM H or W < 1, pitch < W, negative offset, unaligned sse or coef,
 * non-positive frame stride with several frames. */
adct_status adct_jam_evaluate_stream(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                     const adct_plane *planes, int n_planes,
                                     adct_transform_id base, int N, int r, int quant_step,
                                     int32_t *coef, uint8_t *recon, int64_t frame_stride_out,
                                     uint64_t *sse, adct_stream_t stream);

/* ---------------------------------------------------------------- non-orthogonal matrices */

/* Zonal transform coding with an invertible integer matrix T whose rows need
 * not be orthogonal (the signed DCT and BAS-2008b among the paper's
 * competitors, Sec. 2 and 4.3): per 8x8 block B = C_hat A C_hat^T with
 * C_hat = S T, S = diag(1/sqrt(diag(T T^T))), the first r zig-zag coefficients
 * kept, and the inverse decoder A = C_hat^-1 B' C_hat^-T (the transpose inverse
 * of Sec. 6.1.1 holds for orthogonal rows only), rounded half to even and
 * clipped; squared errors per (frame, plane).  The reconstruction equals
 * adj(T) Y' adj(T)^T / det(T)^2 with Y' the kept integer stage and is computed
 * exactly, after adj(T) and det(T) are divided by their common factor (in
 * float32 where that leaves a power-of-two denominator and numerators below
 * 2^24, as for the signed DCT and BAS-2008b; in float64 otherwise).  frames / planes / recon / frame strides as in adct_evaluate_stream
 * (H, W multiples of 8).  T: host int8 [64] row-major.  sse: device uint64
 * [n_frames][n_planes], 8-byte aligned, zeroed by the call then accumulated;
 * recon nullable.  No quantiser (the paper's image experiment is zonal).
 * Errors: ADCT_EINVAL null frames / planes / T / sse, T singular; ADCT_ERANGE r
 * not in [1, 64], n_frames < 1, n_planes not in [1, 4], a plane with H or pitch
 * >= 2^24 or H * pitch >= 2^31, too many blocks;
 * ADCT_EDIM a plane not a positive multiple of 8, pitch < W, negative offset,
 * unaligned sse, non-positive frame stride with several frames; ADCT_EOVERFLOW
 * T whose exact numerators (after the common factor) would pass 2^53, or whose
 * integer stage Y would pass 2^31 / 8. */
adct_status adct_evaluate_inverse(const uint8_t *frames, int64_t frame_stride, int n_frames,
                                  const adct_plane *planes, int n_planes, const int8_t *T, int r,
                                  uint8_t *recon, int64_t frame_stride_out, uint64_t *sse,
                                  adct_stream_t stream);

/* Unified coding gain C_g* (Sec. 4.2.3) of n_t real 8x8 matrices C_hat at n_rho
 * correlations of the first-order Markov model, R_x[i][j] = rho^|i-j| (the curve
 * of Sec. 4.3 is its difference to the exact DCT's): 10 sum_i -log10(A_i B_i)/8,
 * A_i = sum_jk c_ij c_ik rho^|j-k|, B_i the squared norm of row i of C_hat^-1.
 * c_hat: host double [n_t][64] row-major; rho: host double [n_rho] in [0, 1);
 * cg_out: host double [n_t][n_rho] (dB).  Synchronises `stream`; stages in a
 * grow-only device buffer kept between calls (adct_release_caches frees it);
 * calls on one device are serialised.  Errors: ADCT_EINVAL null; ADCT_ERANGE counts
 * below 1, n_t * n_rho > 2^26, rho outside [0, 1). */
adct_status adct_coding_gain_sweep(const double *c_hat, int n_t, const double *rho, int n_rho,
                                   double *cg_out, adct_stream_t stream);

/* The same sweep for callers that cannot allocate device memory (code that must
 * not call hipMalloc, tight serving loops): identical arguments and results,
 * but the device copies of c_hat and rho and the results are staged in a fixed
 * 2 MiB array that each GPU the library runs on holds from the first call until
 * the process ends; no call allocates or frees anything.  Limit:
 * 64 n_t + n_rho + n_t n_rho <= 262,144 (ADCT_ERANGE beyond).  Every call on
 * one GPU stages into the same array: calls that overlap on one GPU (other
 * threads, other streams) race and must be serialised by the caller; the call
 * synchronises `stream` before it returns.  Other errors as above. */
adct_status adct_coding_gain_sweep_noalloc(const double *c_hat, int n_t, const double *rho, int n_rho,
                                           double *cg_out, adct_stream_t stream);

/* ---------------------------------------------------------------- search */

/* Search modes of adct_derive_transform (Sec. 3.5 and 4.1).  Exact ties in
 * angle are real (scalar multiples, mirror images, equal irrational angles):
 *   CLOSURE    every matrix reachable under any resolution of the exact ties
 *              (cosines within 1e-12 are tied; groups by single linkage)
 *   CANONICAL  one matrix per order: among tied candidates the smaller
 *              squared norm, then the smaller canonical index */
typedef enum { ADCT_SEARCH_CLOSURE = 0, ADCT_SEARCH_CANONICAL = 1 } adct_search_mode;

/* Greedy angle-similarity search (Eq. (6), the algorithm of Sec. 3.5): for each
 * row order, each row k in turn takes the candidate of D = P^8 \ {0} with the
 * smallest angle to DCT row k among those orthogonal to every row chosen so
 * far; an order whose feasible set empties is dead.
 *   P, nP         host: the entry set (distinct values in [-8, 8], must hold 0;
 *                 the extended sets of Sec. 4.1 reach +-8),
 *                 1 <= nP <= 9.  The canonical index of a vector is its
 *                 odometer rank over P ordered 0, 1, -1, 2, -2, ... (first
 *                 coordinate most significant).
 *   orders        host: n_orders x n_free row indices (0-based) of the free
 *                 rows, or NULL for all orders of the free rows
 *   fix_rows_1_5  nonzero: rows 1 and 5 (indices 0 and 4) are fixed to
 *                 [1]*8 and [1,-1,-1,1,1,-1,-1,1] (Sec. 4.1) and the other six
 *                 rows are free (720 orders); zero: all 8 rows free
 *   out, cap_out  host: the distinct matrices found, sorted by their 64 bytes
 *   n_out         host: number of distinct matrices (also when > cap_out,
 *                 which returns ADCT_ECAP after filling cap_out)
 *   angles_out    host, nullable: cap_out x 8 angles (radians) of each row to
 *                 the matching DCT row
 *   leaves_out, dead_out  host, nullable: completed and dead (order, tie
 *                 branch) paths
 * Each search state keeps its feasible list (space indices, 4 bytes each) on the
 * device for one depth; ADCT_ERANGE if a depth's lists would pass 32 GB.
 * Synchronises `stream`.  The enumerated space lives in grow-only device buffers
 * kept per device until the process ends; searches on one device take a lock
 * and run one at a time (this and adct_search_topk). */
adct_status adct_derive_transform(const int8_t *P, int nP, int mode, const uint8_t *orders,
                                  int n_orders, int fix_rows_1_5, adct_matrix *out, int cap_out,
                                  int *n_out, double *angles_out, int64_t *leaves_out,
                                  int64_t *dead_out, adct_stream_t stream);

/* Top-k form of the row search (Sec. 3.3 objective over the whole space, one
 * list per DCT row): for each row r the k candidates of P^8 \ {0} with the
 * smallest angle, ranked by cosine tie groups (1e-12), then squared norm, then
 * canonical index.  primitive != 0 keeps only vectors whose entries have gcd 1
 * (a positive multiple of a row gives the same normalised row).
 *   vec_out  host int8 [8][k][8];  idx_out host [8][k] canonical indices;
 *   cos_out  host [8][k].  Synchronises `stream`; shares the per-device search
 *   buffers and lock of adct_derive_transform. */
adct_status adct_search_topk(const int8_t *P, int nP, int k, int primitive, int8_t *vec_out,
                             int64_t *idx_out, double *cos_out, adct_stream_t stream);

/* Every choice of one vector per row list whose 8 vectors are pairwise
 * orthogonal (T T^T diagonal, Sec. 3.4), in lexicographic order of positions.
 *   lists  host int8: the 8 lists concatenated, list r has len[r] vectors of 8
 *   out    host int32 [cap][8] positions;  n_total  host: number of tuples (all
 *          of them, even beyond cap).  Synchronises `stream`. */
adct_status adct_orthogonal_tuples(const int8_t *lists, const int *len, int32_t *out, int64_t cap,
                                   int64_t *n_total, adct_stream_t stream);

/* ---------------------------------------------------------------- batch */

/* Rate-distortion sweep over many images (Sec. 6.1.1: per-image MSE / PSNR for
 * each retained count r, averaged over an image set, for the exact DCT and the
 * approximations).  For every image i, transform t and r in [r_lo, r_hi]:
 * sse[(i * n_transforms + t) * (r_hi - r_lo + 1) + (r - r_lo)] = sum of
 * squared errors of the rounded, clipped reconstruction (integer transforms:
 * exact; ADCT_DCT: float64).  images[i] describes image i inside the device
 * buffer `base` (offset, H, W, pitch; all multiples of 8).  Up to 64 images and
 * 8 transforms (ADCT_DCT .. ADCT_T4) per call.  sse: device uint64, zeroed by
 * the call.  The whole sweep is one persistent launch; wgs_per_cu (1..16)
 * resident single-wave workgroups per compute unit; split (1..n_transforms)
 * transform groups per 64-block tile. */
adct_status adct_evaluate_batch(const uint8_t *base, const adct_plane *images, int n_images,
                                const adct_transform_id *transforms, int n_transforms, int r_lo,
                                int r_hi, uint64_t *sse, int wgs_per_cu, int split,
                                adct_stream_t stream);

/* A prepared sweep: the same computation with its schedule picked by timing
 * every candidate (wgs_per_cu, split, and the DCT kernel's workgroups per CU)
 * on the given input when autotune != 0 (this runs the sweep several times on
 * `stream` and synchronises it).  The plan owns a second stream, two events and
 * two device work counters (8 bytes); when the list holds both the DCT and
 * integer transforms, a launch runs the DCT kernel on that second stream beside
 * the integer kernel on `stream` (forked after the zero fill, joined back into
 * `stream` before the call's work counts as done), and both kernels take their
 * items from the counters.  Launches of one plan are ordered by `stream`: two
 * launches of the same plan that overlap on the device (on different streams)
 * race on its counters and on sse.  The call is capturable into a HIP graph.
 * All pointers are kept: the buffers must outlive the plan.  Destroying the
 * plan waits for its second stream; the caller's stream must have finished
 * the plan's launches. */
typedef struct adct_batch_plan_s *adct_batch_plan;
adct_status adct_batch_plan_create(const uint8_t *base, const adct_plane *images, int n_images,
                                   const adct_transform_id *transforms, int n_transforms, int r_lo,
                                   int r_hi, uint64_t *sse, int autotune, adct_batch_plan *out,
                                   adct_stream_t stream);
adct_status adct_batch_plan_launch(adct_batch_plan plan, adct_stream_t stream);
adct_status adct_batch_plan_info(adct_batch_plan plan, int *wgs_per_cu, int *split, double *tuned_ms);
adct_status adct_batch_plan_destroy(adct_batch_plan plan);

/* ---------------------------------------------------------------- learned post-filter
 *
 * Not part of the paper's method: a small network applied after decoding that
 * removes part of the coding error the approximation leaves.  On a decoded
 * 8-bit image x (one plane):
 *   xn = (x - 128) / 64
 *   a1 = relu(conv3x3(xn; W1, b1))   1 -> 32 channels
 *   a2 = relu(conv3x3(a1; W2, b2))   32 -> 32
 *   y  = xn + conv3x3(a2; W3, b3)    32 -> 1
 *   output pixel = clip(round_half_even(128 + 64 y), 0, 255)
 * Each 3x3 convolution is a cross-correlation that zero-pads its own input.
 * Weights and activations enter the matrix cores as bfloat16 (round to
 * nearest even), accumulation is float32, biases stay float32.
 *
 * Parameters: one flat float32 device vector of ADCT_FILTER_PARAMS values in
 * PyTorch Conv2d order: W1 (32,1,3,3), b1 (32), W2 (32,32,3,3), b2 (32),
 * W3 (1,32,3,3), b3 (1).  Training minimises the mean over all pixels of
 * (y - (orig - 128) / 64)^2; gradients are taken with respect to the bfloat16
 * weights, with the loss gradient and the masked input gradients rounded to
 * bfloat16 where they enter the matrix cores.  All buffers are caller-owned
 * device memory; calls enqueue on `stream` and do not synchronise. */
#define ADCT_FILTER_PARAMS 9857

/* Bytes of the packed form of the weights (operand order of the kernels). */
int64_t adct_filter_packed_bytes(void);

/* Packs params (device float32[ADCT_FILTER_PARAMS]) into `packed` (device,
 * adct_filter_packed_bytes(), 16-byte aligned): bfloat16 weights in operand
 * order plus the float32 biases.  The packed form is what adct_filter_apply reads. */
adct_status adct_filter_pack(const float *params, void *packed, adct_stream_t stream);

/* Workspace bytes adct_filter_grad / adct_filter_train_step need for n images
 * of H x W (H a multiple of 16, W = 32 or 64); -1 when the shape is not
 * supported. */
int64_t adct_filter_workspace_bytes(int n, int H, int W);

/* Loss and gradient on a batch.  recon, orig: device uint8 [n][H][W]
 * (contiguous) decoded and original images.  grad: device float32
 * [ADCT_FILTER_PARAMS] (overwritten); loss: device float32 scalar (nullable);
 * y_out: device float32 [n][H][W] network output y (nullable).  The sums over
 * pixels run in a fixed order, so repeated calls give identical results.
 * Errors: ADCT_EINVAL null pointer, ADCT_EDIM unsupported shape, ADCT_ECAP
 * workspace smaller than adct_filter_workspace_bytes. */
adct_status adct_filter_grad(const float *params, const uint8_t *recon, const uint8_t *orig, int n, int H, int W,
                             void *workspace, int64_t ws_bytes, float *grad, float *loss, float *y_out,
                             adct_stream_t stream);

/* One Adam step (Kingma and Ba, bias-corrected; `step` counts from 1) on
 * params with moment buffers m and v (device float32[ADCT_FILTER_PARAMS], zero
 * before the first step), in float32.  Errors: ADCT_ERANGE step < 1, lr < 0,
 * beta outside [0, 1), eps <= 0. */
adct_status adct_filter_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                             float beta1, float beta2, float eps, adct_stream_t stream);

/* adct_filter_grad (gradient kept in the workspace) followed by adct_filter_adam. */
adct_status adct_filter_train_step(float *params, float *m, float *v, int step, float lr, float beta1, float beta2,
                                   float eps, const uint8_t *recon, const uint8_t *orig, int n, int H, int W,
                                   void *workspace, int64_t ws_bytes, float *loss, adct_stream_t stream);

/* Inference on decoded frames: out = filter(frames), every plane of every
 * frame, all three layers in one kernel without writing activations.  Planes
 * as in adct_evaluate_stream (any H, W >= 1, pitch >= W); frames, out and
 * orig use the same plane offsets and pitches with their own frame strides.
 * out must not alias frames.  When sse (device uint64 [n_frames][n_planes],
 * zeroed by the call) is given, it receives the squared error of out against
 * orig.  Errors: ADCT_EINVAL null pointer / aliasing / sse without orig,
 * ADCT_EDIM plane geometry or unaligned packed weights. */
adct_status adct_filter_apply(const void *packed, const uint8_t *frames, int64_t frame_stride, int n_frames,
                              const adct_plane *planes, int n_planes, uint8_t *out, int64_t frame_stride_out,
                              const uint8_t *orig, int64_t frame_stride_orig, uint64_t *sse,
                              adct_stream_t stream);

/* Keep rule and fallback.  Frame f keeps its filtered planes (already in out)
 * when the sum over planes of sse_filtered[f] is not larger than that of
 * sse_reference[f] (same samples, so: PSNR at least the reference's, e.g. the
 * exact DCT at the same r and quantiser); otherwise the plain reconstruction
 * `plain` is copied into out.  keep (device uint8 [n_frames], nullable)
 * receives the decision.  Plane W, pitch, offsets, strides and buffers must be
 * multiples of 8 bytes (ADCT_EDIM). */
adct_status adct_filter_select(const uint64_t *sse_filtered, const uint64_t *sse_reference, int n_frames,
                               int n_planes, const uint8_t *plain, int64_t frame_stride_plain,
                               const adct_plane *planes, uint8_t *out, int64_t frame_stride_out, uint8_t *keep,
                               adct_stream_t stream);

/* Checkpoint and resume of the post-filter (for callers that train, stop and
 * continue, or ship trained weights): a self-checking host byte blob holding a
 * 64-byte header (magic "ADCTFILT", format version 1, parameter count 9,857, a
 * flag for the Adam moments, the Adam step, an FNV-1a 64-bit hash of the
 * payload) and the float32 parameters, optionally followed by the moments m and
 * v.  adct_filter_checkpoint_bytes(with_moments) is the blob size.
 *   save: params (and m, v: both or neither, nullable) device float32 [9857];
 *         blob host, blob_bytes at least the size (ADCT_ECAP); synchronises.
 *   load: validates the whole blob on the host before any copy (ADCT_EINVAL for
 *         a wrong magic, version, count or hash, or moments asked of a blob
 *         without them; ADCT_EDIM for a size that does not match its header),
 *         then fills params (and m, v when given) and *step (nullable);
 *         synchronises. */
int64_t adct_filter_checkpoint_bytes(int with_moments);
adct_status adct_filter_save(const float *params, const float *m, const float *v, int step, void *blob,
                             int64_t blob_bytes, adct_stream_t stream);
adct_status adct_filter_load(const void *blob, int64_t blob_bytes, float *params, float *m, float *v, int *step,
                             adct_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ADCT_H */
