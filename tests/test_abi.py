"""The C ABI library loads, exports every declared symbol, and validates its
arguments on the host (no GPU work is started by any call here)."""

import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import codec as Co
from oracle import matrices as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(adct_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    lib = A.lib()
    names = _declared()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("name", ["T1", "T2", "LO", "T6", "RDCT", "T4"])
def test_builtin_matrices_match_oracle(name):
    assert np.array_equal(A.matrix_get(name), M.TRANSFORMS[name])


def test_forward_bound_matches_interval_propagation():
    assert A.transform_bounds("T1", 10)[0] == 18360
    assert A.transform_bounds("LO", 10)[0] == 65280


@pytest.mark.parametrize("name,r", [("T1", 10), ("T1", 3), ("RDCT", 10), ("LO", 21)])
def test_inverse_bound_is_attained(name, r):
    # the library's bound on the exact inverse numerator is the maximum over
    # 8-bit blocks: the extremal block (255 where the kernel is positive, 0
    # elsewhere) reaches it in the oracle's exact inverse
    t = M.TRANSFORMS[name]
    bound = A.transform_bounds(name, r)[1]
    n = M.row_norms2(t)
    best = 0
    mask = Co.zonal_mask(r)
    for x in range(8):
        for y in range(8):
            for sign in (1, -1):
                # sign pattern of d num(x, y) / d A(u, v)
                e = np.zeros((64, 8, 8), dtype=np.int64)
                for u in range(8):
                    for v in range(8):
                        e[8 * u + v, u, v] = 1
                yk = Co.forward_int(e, t) * mask
                num, _ = Co.inverse_exact(yk, t)
                g = num[:, x, y]
                blk = np.where(sign * g > 0, 255, 0).reshape(1, 8, 8)
                yy = Co.forward_int(blk, t) * mask
                nn, _ = Co.inverse_exact(yy, t)
                best = max(best, abs(int(nn[0, x, y])))
    assert best == bound


def test_bounds_are_memoised_consistently():
    """The library keeps the last few exact bounds per thread, keyed by the
    matrix bytes and r: more distinct (matrix, r) pairs than it keeps, asked in
    an interleaved order (so entries are evicted and refilled), always give
    the values of the first asking; a caller matrix equal to a built-in one
    shares its entries, and a matrix differing in one entry does not."""
    keys = [(name, r) for name in ("T1", "T2", "LO", "T6", "RDCT", "T4") for r in (3, 10)]
    first = {k: A.transform_bounds(*k) for k in keys}
    for rep in range(3):
        for k in (keys[rep::3] + keys[::-1]):
            assert A.transform_bounds(*k) == first[k], k
    t1 = np.array(M.T1, dtype=np.int64)
    assert A.transform_bounds("CUSTOM", 10, custom=t1) == first[("T1", 10)]
    t1b = t1.copy()
    t1b[0] *= 2                               # another matrix (row 0 doubled): other bounds
    fb, ib = A.transform_bounds("CUSTOM", 10, custom=t1b)
    assert (fb, ib) != first[("T1", 10)] and fb == 4 * 255 * 64   # Y[0][0] of a block of 255s
    assert A.transform_bounds("T1", 10) == first[("T1", 10)]


def _call(fn, *args):
    return getattr(A.lib(), fn)(*args)


FAKE = ctypes.c_void_p(4096)          # never dereferenced: every case fails validation


@pytest.mark.parametrize("args,expect", [
    ((None, 8, 8, 8, A.T1, None, 10, 0, FAKE, None, None), -1),         # null image
    ((FAKE, 8, 8, 8, A.T1, None, 10, 0, None, None, None), -1),         # no output
    ((FAKE, 12, 8, 8, A.T1, None, 10, 0, FAKE, None, None), -2),        # H % 8
    ((FAKE, 8, 16, 8, A.T1, None, 10, 0, FAKE, None, None), -2),        # pitch < W
    ((FAKE, 8, 8, 12, A.T1, None, 10, 0, FAKE, None, None), -2),        # pitch % 8
    ((FAKE, 8, 8, 8, A.T1, None, 0, 0, FAKE, None, None), -3),          # r = 0
    ((FAKE, 8, 8, 8, A.T1, None, 65, 0, FAKE, None, None), -3),         # r = 65
    ((FAKE, 8, 8, 8, A.T1, None, 10, -1, FAKE, None, None), -3),        # step < 0
    ((FAKE, 8, 8, 8, A.LO, None, 10, 0, FAKE, None, None), -4),         # LO into int16
    ((FAKE, 8, 8, 8, 42, None, 10, 0, FAKE, None, None), -1),           # unknown id
])
def test_encode_argument_errors(args, expect):
    assert _call("adct_encode_blocks", *args) == expect
    assert A.lib().adct_last_error()


def test_stream_argument_errors():
    planes = A.planes_struct([(0, 16, 16, 16)])
    sse = ctypes.c_void_p(8192)
    lib = A.lib()
    assert lib.adct_evaluate_stream(FAKE, 256, 0, planes, 1, A.T1, None, 10, 0, None, None, 0, sse, None) == -3
    assert lib.adct_evaluate_stream(FAKE, 256, 1, planes, 5, A.T1, None, 10, 0, None, None, 0, sse, None) == -3
    assert lib.adct_evaluate_stream(FAKE, 256, 1, planes, 1, A.T1, None, 10, 0, None, None, 0, None, None) == -1
    bad = A.planes_struct([(4, 16, 16, 16)])
    assert lib.adct_evaluate_stream(FAKE, 256, 1, bad, 1, A.T1, None, 10, 0, None, None, 0, sse, None) == -2


def test_bandwidth_probe_argument_errors():
    planes = A.planes_struct([(0, 16, 16, 16)])
    lib = A.lib()
    assert lib.adct_stream_bandwidth_probe(None, 256, 1, planes, 1, 10, None, None, 0, None) == -1
    assert lib.adct_stream_bandwidth_probe(FAKE, 256, 0, planes, 1, 10, None, None, 0, None) == -3
    assert lib.adct_stream_bandwidth_probe(FAKE, 256, 1, planes, 1, 0, None, None, 0, None) == -3
    bad = A.planes_struct([(4, 16, 16, 16)])
    assert lib.adct_stream_bandwidth_probe(FAKE, 256, 1, bad, 1, 10, None, None, 0, None) == -2


def test_plane_height_bound():
    """Row offsets are formed with 24-bit multiplies, so planes of 2^24 rows or
    more are refused (ADCT_EDIM) before any device work."""
    big = A.planes_struct([(0, 1 << 24, 8, 8)])
    sse = ctypes.c_void_p(8192)
    assert A.lib().adct_evaluate_stream(FAKE, 0, 1, big, 1, A.T1, None, 10, 0, None, None, 0, sse, None) == -2


def test_quantiser_steps_accepted():
    """Tie-free steps and steps that admit exact halves (decided exactly in the
    field of the row norms' square roots) are both accepted for every built-in
    matrix, at the zonal bands of r = 10 and r = 64, up to the largest step."""
    lib = A.lib()
    for tid, step in [(A.T1, 8), (A.T1, 16), (A.T1, 24), (A.T4, 8), (A.T6, 40), (A.LO, 32),
                      (A.T1, 4), (A.T1, 5), (A.T2, 20), (A.LO, 16), (A.RDCT, 6), (A.T6, 3), (A.T4, 1)]:
        for r in (10, 64):
            assert lib.adct_check_codec_args(tid, None, r, step, 1) == 0, (tid, step, r)
    for tid in (A.T1, A.T2, A.LO, A.T6, A.RDCT, A.T4):
        assert lib.adct_check_codec_args(tid, None, 64, 65535, 1) == 0
        assert lib.adct_check_codec_args(tid, None, 64, 65533, 1) == 0
    assert lib.adct_check_codec_args(A.LO, None, 10, 0, 1) == -4
    assert lib.adct_check_codec_args(A.LO, None, 10, 0, 0) == 0


def test_three_independent_roots_refused():
    """Row norms (2, 2, 3, 2, 6, 5, 5, 1) bring in sqrt 2, sqrt 3 and sqrt 5:
    with a step that admits exact halves the full band (r = 64) cannot be
    decided with two generators (ADCT_ENOTSUP); the band of r = 10 only meets
    sqrt 6, and tie-free steps need no decision."""
    t = np.zeros((8, 8), dtype=np.int64)
    t[0:2, 0:2] = [[1, 1], [1, -1]]
    t[2:5, 2:5] = [[1, 1, 1], [1, -1, 0], [1, 1, -2]]
    t[5:7, 5:7] = [[1, 2], [2, -1]]
    t[7, 7] = 1
    m = A._matrix_struct(t)
    n = [int(v) for v in np.diag(t @ t.T)]
    assert n == [2, 2, 3, 2, 6, 5, 5, 1], n
    lib = A.lib()
    assert lib.adct_check_codec_args(A.CUSTOM, m, 64, 1, 0) == -7
    assert lib.adct_check_codec_args(A.CUSTOM, m, 10, 1, 0) == 0
    assert lib.adct_check_codec_args(A.CUSTOM, m, 64, 0, 0) == 0


def test_custom_matrix_validation_host_only():
    """ADCT_CUSTOM takes any int8 matrix with orthogonal rows: the caller's n must
    be diag(T T^T); a missing matrix, non-orthogonal rows or a wrong n are
    ADCT_EINVAL; the quantiser steps and the int16 bound work as for the
    built-in matrices."""
    lib = A.lib()
    m = A._matrix_struct(M.T1)
    assert lib.adct_check_codec_args(A.CUSTOM, m, 10, 0, 1) == 0
    assert lib.adct_check_codec_args(A.CUSTOM, m, 10, 16, 1) == 0
    assert lib.adct_check_codec_args(A.CUSTOM, m, 10, 12, 1) == 0       # ties decided exactly
    assert lib.adct_check_codec_args(A.CUSTOM, None, 10, 0, 1) == -1
    bad_n = A._matrix_struct(M.T1)
    bad_n.n[2] += 1
    assert lib.adct_check_codec_args(A.CUSTOM, bad_n, 10, 0, 1) == -1
    skew = M.T1.copy()
    skew[1, 0] += 1
    assert lib.adct_check_codec_args(A.CUSTOM, A._matrix_struct(skew), 10, 0, 1) == -1
    assert lib.adct_check_codec_args(A.CUSTOM, A._matrix_struct(M.t_sdct()), 10, 0, 1) == -1
    zero_row = M.T1.copy()
    zero_row[7] = 0
    assert lib.adct_check_codec_args(A.CUSTOM, A._matrix_struct(zero_row), 10, 0, 1) == -1
    lo = A._matrix_struct(M.T_LO_X2)
    assert lib.adct_check_codec_args(A.CUSTOM, lo, 10, 0, 1) == -4      # int16 output
    assert lib.adct_check_codec_args(A.CUSTOM, lo, 10, 0, 0) == 0
    assert lib.adct_check_codec_args(A.CUSTOM, lo, 10, 32, 1) == 0
    # entries up to +-127 with orthogonal rows: a scaled Hadamard-like matrix
    big = np.array([[1, 1], [1, -1]])
    h8 = np.kron(np.kron(big, big), big) * 127
    assert lib.adct_check_codec_args(A.CUSTOM, A._matrix_struct(h8), 64, 0, 0) == 0
    assert lib.adct_check_codec_args(A.CUSTOM, A._matrix_struct(h8), 64, 16, 0) == -3   # |Y| >= 2^24


def test_decode_float_coefficients_host_only():
    lib = A.lib()
    # exactly one of coef_int / coef_scaled; float B takes no quantiser step
    assert lib.adct_decode_blocks(FAKE, FAKE, 8, 8, FAKE, 8, A.T1, None, 10, 0, None) == -1
    assert lib.adct_decode_blocks(None, FAKE, 8, 8, FAKE, 8, A.T1, None, 10, 16, None) == -1
    assert lib.adct_decode_blocks(None, FAKE, 8, 8, FAKE, 8, A.CUSTOM, None, 10, 0, None) == -1


def test_search_argument_errors_host_only():
    lib = A.lib()
    n = ctypes.c_int()
    out = (A.Matrix * 4)()
    bad_p = (ctypes.c_int8 * 2)(1, -1)                       # no zero
    assert lib.adct_derive_transform(ctypes.cast(bad_p, ctypes.c_void_p), 2, 0, None, 0, 1, out, 4,
                                     ctypes.byref(n), None, None, None, None) == -1
    rep = (ctypes.c_int8 * 3)(0, 1, 1)                       # repeated entry
    assert lib.adct_derive_transform(ctypes.cast(rep, ctypes.c_void_p), 3, 0, None, 0, 1, out, 4,
                                     ctypes.byref(n), None, None, None, None) == -1
    big = (ctypes.c_int8 * 3)(0, 1, 9)                       # entry beyond +-8
    assert lib.adct_derive_transform(ctypes.cast(big, ctypes.c_void_p), 3, 0, None, 0, 1, out, 4,
                                     ctypes.byref(n), None, None, None, None) == -3
    p1 = (ctypes.c_int8 * 3)(0, 1, -1)
    assert lib.adct_derive_transform(ctypes.cast(p1, ctypes.c_void_p), 3, 7, None, 0, 1, out, 4,
                                     ctypes.byref(n), None, None, None, None) == -1   # bad mode
    orders = (ctypes.c_uint8 * 6)(1, 2, 3, 5, 6, 6)
    assert lib.adct_derive_transform(ctypes.cast(p1, ctypes.c_void_p), 3, 0,
                                     ctypes.cast(orders, ctypes.c_void_p), 1, 1, out, 4,
                                     ctypes.byref(n), None, None, None, None) == -1
    assert lib.adct_search_topk(ctypes.cast(p1, ctypes.c_void_p), 3, 0, 1, FAKE, FAKE, FAKE, None) == -3


def test_filter_argument_errors_host_only():
    """Every filter entry point validates before any device work: empty
    batches, unsupported shapes, small workspaces, bad optimiser settings,
    aliasing and plane geometry."""
    lib = A.lib()
    F2 = ctypes.c_void_p(8192)
    assert lib.adct_filter_packed_bytes() > 20992 * 2
    assert lib.adct_filter_workspace_bytes(2, 64, 64) > 0
    for n, h, w in [(0, 64, 64), (2, 40, 64), (2, 64, 48), (2, 64, 128), (2, 0, 64)]:
        assert lib.adct_filter_workspace_bytes(n, h, w) == -1, (n, h, w)
    need = lib.adct_filter_workspace_bytes(2, 32, 64)
    assert lib.adct_filter_grad(FAKE, FAKE, F2, 0, 32, 64, FAKE, need, FAKE, None, None, None) == -3
    assert lib.adct_filter_grad(FAKE, FAKE, F2, 2, 32, 48, FAKE, need, FAKE, None, None, None) == -2
    assert lib.adct_filter_grad(FAKE, FAKE, F2, 2, 32, 64, FAKE, need - 1, FAKE, None, None, None) == -5
    assert lib.adct_filter_grad(None, FAKE, F2, 2, 32, 64, FAKE, need, FAKE, None, None, None) == -1
    for step, lr, b1, b2, eps in [(0, 1e-3, 0.9, 0.999, 1e-8), (1, -1.0, 0.9, 0.999, 1e-8),
                                  (1, 1e-3, 1.0, 0.999, 1e-8), (1, 1e-3, 0.9, 0.999, 0.0)]:
        assert lib.adct_filter_adam(FAKE, FAKE, FAKE, FAKE, step, lr, b1, b2, eps, None) == -3
    planes = A.planes_struct([(0, 16, 16, 16)])
    assert lib.adct_filter_apply(FAKE, FAKE, 256, 0, planes, 1, F2, 256, None, 0, None, None) == -3
    assert lib.adct_filter_apply(FAKE, FAKE, 256, 1, planes, 5, F2, 256, None, 0, None, None) == -3
    assert lib.adct_filter_apply(FAKE, FAKE, 256, 1, planes, 1, FAKE, 256, None, 0, None, None) == -1
    assert lib.adct_filter_apply(FAKE, FAKE, 256, 1, planes, 1, F2, 256, None, 0, F2, None) == -1
    assert lib.adct_filter_apply(ctypes.c_void_p(4100), FAKE, 256, 1, planes, 1, F2, 256, None, 0,
                                 None, None) == -2
    bad = A.planes_struct([(0, 16, 16, 15)])                       # pitch < W
    assert lib.adct_filter_apply(FAKE, FAKE, 256, 1, bad, 1, F2, 256, None, 0, None, None) == -2
    odd = A.planes_struct([(0, 16, 12, 16)])                       # select copies 8-byte words
    assert lib.adct_filter_select(FAKE, FAKE, 1, 1, FAKE, 256, odd, F2, 256, None, None) == -2
    assert lib.adct_filter_select(FAKE, FAKE, 0, 1, FAKE, 256, planes, F2, 256, None, None) == -3


def test_batch_empty_and_oversized_sets():
    lib = A.lib()
    planes = A.planes_struct([(0, 16, 16, 16)])
    tids = (ctypes.c_int * 1)(A.T1)
    assert lib.adct_evaluate_batch(FAKE, planes, 0, tids, 1, 1, 63, FAKE, 4, 1, None) == -3
    assert lib.adct_evaluate_batch(FAKE, planes, 1, tids, 0, 1, 63, FAKE, 4, 1, None) == -3


def test_ssim_argument_errors_host_only():
    """adct_ssim validates every argument before it launches anything."""
    lib = A.lib()
    FAKE = ctypes.c_void_p(4096)
    OUT = ctypes.c_void_p(8192)
    ok = A.planes_struct([(0, 32, 32, 32)])
    assert lib.adct_ssim(None, 0, FAKE, 0, 1, ok, 1, OUT, None) == -1
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, ok, 1, None, None) == -1
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 0, ok, 1, OUT, None) == -3
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, ok, 0, OUT, None) == -3
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, ok, 5, OUT, None) == -3
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, A.planes_struct([(0, 10, 32, 32)]), 1, OUT, None) == -2
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, A.planes_struct([(0, 32, 10, 32)]), 1, OUT, None) == -2
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, A.planes_struct([(0, 32, 32, 16)]), 1, OUT, None) == -2
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, ok, 1, ctypes.c_void_p(8196), None) == -2
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 2, ok, 1, OUT, None) == -2
    assert lib.adct_ssim(FAKE, 0, FAKE, 0, 1, A.planes_struct([(0, 1 << 14, 1 << 13, 1 << 13)]), 1, OUT,
                         None) == -3


def test_jam_matrix_host_only():
    """adct_jam_matrix (host only) returns the oracle's 16- and 32-point matrices."""
    from oracle import jam
    from oracle import matrices as M
    for n in (16, 32):
        t, nr = A.jam_matrix(n)
        want = jam.jam_n(M.T1, n)
        assert np.array_equal(t.astype(np.int64), want)
        assert np.array_equal(nr.astype(np.int64), np.sum(want * want, axis=1))
    lib = A.lib()
    buf = (ctypes.c_int8 * 1024)()
    nb = (ctypes.c_int32 * 32)()
    assert lib.adct_jam_matrix(A.TRANSFORM_IDS["T1"], 8, buf, nb) == -3
    assert lib.adct_jam_matrix(A.TRANSFORM_IDS["LO"], 16, buf, nb) == -7
    assert lib.adct_jam_matrix(A.TRANSFORM_IDS["T1"], 16, None, nb) == -1


def test_jam_argument_errors_host_only():
    """adct_jam_evaluate_stream validates every argument before it launches anything."""
    lib = A.lib()
    FAKE = ctypes.c_void_p(4096)
    SSE = ctypes.c_void_p(8192)
    T1 = A.TRANSFORM_IDS["T1"]
    ok = A.planes_struct([(0, 40, 40, 40)])

    def call(frames=FAKE, fs=0, nf=1, planes=ok, npl=1, base=T1, n=16, r=10, step=16, coef=None,
             sse=SSE):
        return lib.adct_jam_evaluate_stream(frames, fs, nf, planes, npl, base, n, r, step, coef, None,
                                            0, sse, None)
    assert call(frames=None) == -1
    assert call(sse=None) == -1
    assert call(base=A.TRANSFORM_IDS["T6"]) == -7
    assert call(n=8) == -3 and call(n=64) == -3
    assert call(r=0) == -3 and call(r=257) == -3 and call(n=32, r=1025) == -3
    assert call(step=-16) == -3 and call(step=4112) == -3
    assert call(step=8) == -7 and call(n=32, step=16) == -7
    assert call(nf=0) == -3
    assert call(npl=0) == -3 and call(npl=5) == -3
    assert call(nf=2, fs=0) == -2
    assert call(planes=A.planes_struct([(0, 0, 40, 40)])) == -2
    assert call(planes=A.planes_struct([(0, 40, 40, 39)])) == -2
    assert call(planes=A.planes_struct([(-1, 40, 40, 40)])) == -2
    assert call(sse=ctypes.c_void_p(8196)) == -2
    assert call(coef=ctypes.c_void_p(4098)) == -2
    # 32-bit in-plane offsets: H and pitch below 2^24, the plane below 2^31 bytes
    assert call(planes=A.planes_struct([(0, 1 << 24, 40, 40)])) == -3
    assert call(planes=A.planes_struct([(0, 40, 40, 1 << 24)])) == -3
    assert call(planes=A.planes_struct([(0, 1 << 17, 40, 1 << 14)])) == -3


def test_inverse_codec_argument_errors_host_only():
    """adct_evaluate_inverse validates every argument before it launches anything."""
    lib = A.lib()
    FAKE = ctypes.c_void_p(4096)
    SSE = ctypes.c_void_p(8192)
    ok = A.planes_struct([(0, 16, 16, 16)])
    good = (ctypes.c_int8 * 64)(*[int(v) for v in np.sign(np.cos(np.outer(np.arange(8), 2 * np.arange(8) + 1)
                                                                   * np.pi / 16)).ravel()])
    sing = (ctypes.c_int8 * 64)(*([1] * 64))

    def call(frames=FAKE, nf=1, planes=ok, npl=1, T=good, r=10, sse=SSE, fs=0):
        return lib.adct_evaluate_inverse(frames, fs, nf, planes, npl, ctypes.cast(T, ctypes.c_void_p) if T else None,
                                         r, None, 0, sse, None)
    assert call(frames=None) == -1 and call(T=None) == -1 and call(sse=None) == -1
    assert call(T=sing) == -1
    assert call(r=0) == -3 and call(r=65) == -3
    assert call(nf=0) == -3 and call(npl=0) == -3 and call(npl=5) == -3
    assert call(planes=A.planes_struct([(0, 12, 16, 16)])) == -2
    assert call(planes=A.planes_struct([(0, 16, 16, 8)])) == -2
    assert call(sse=ctypes.c_void_p(8196)) == -2
    assert call(nf=2, fs=0) == -2
    h = np.array([[1]])
    for _ in range(3):
        h = np.block([[h, h], [h, -h]])                        # 8 x 8 Hadamard
    big = (ctypes.c_int8 * 64)(*[int(v) for v in (127 * h).ravel()])   # Y passes 2^31 / 8
    assert call(T=big) == -4
    # 32-bit in-plane offsets: H and pitch below 2^24, the plane below 2^31 bytes
    assert call(planes=A.planes_struct([(0, 1 << 24, 16, 16)])) == -3
    assert call(planes=A.planes_struct([(0, 16, 16, 1 << 24)])) == -3
    assert call(planes=A.planes_struct([(0, 1 << 17, 16, 1 << 14)])) == -3


def test_coding_gain_argument_errors_host_only():
    lib = A.lib()
    c = np.eye(8).ravel()
    rho = np.array([0.5, 1.0])
    out = np.zeros(2)
    assert lib.adct_coding_gain_sweep(None, 1, rho.ctypes.data, 1, out.ctypes.data, None) == -1
    assert lib.adct_coding_gain_sweep(c.ctypes.data, 0, rho.ctypes.data, 1, out.ctypes.data, None) == -3
    assert lib.adct_coding_gain_sweep(c.ctypes.data, 1, rho.ctypes.data, 2, out.ctypes.data, None) == -3


def test_filter_checkpoint_validation_host_only():
    """adct_filter_load checks the whole blob on the host before any copy."""
    import struct
    lib = A.lib()
    n1, n3 = lib.adct_filter_checkpoint_bytes(0), lib.adct_filter_checkpoint_bytes(1)
    assert n1 == 64 + 9857 * 4 and n3 == 64 + 3 * 9857 * 4
    FAKE = ctypes.c_void_p(4096)

    def blob(magic=b"ADCTFILT", version=1, count=9857, flags=0, payload=None, size=None):
        payload = bytes(9857 * 4 * (3 if flags else 1)) if payload is None else payload
        h = 1469598103934665603
        for byte in payload:                                   # FNV-1a 64
            h = ((h ^ byte) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
        head = magic + struct.pack("<IIIiQ", version, count, flags, 7, h) + bytes(32)
        b = head + payload
        return b if size is None else b[:size]

    def load(b, m=None):
        buf = ctypes.create_string_buffer(b, len(b))
        return lib.adct_filter_load(ctypes.cast(buf, ctypes.c_void_p), len(b), FAKE, m, m, None, None)
    assert load(blob(magic=b"NOTAFILT")) == -1
    assert load(blob(version=2)) == -1
    assert load(blob(count=100)) == -1
    assert load(blob(size=n1 - 4)) == -2
    assert load(blob()[:32]) == -2
    good = bytearray(blob())
    good[100] ^= 1                                             # corrupt one payload byte
    assert load(bytes(good)) == -1
    assert load(blob(), m=FAKE) == -1                          # moments asked, none stored
    assert lib.adct_filter_save(None, None, None, 0, FAKE, n1, None) == -1
    assert lib.adct_filter_save(FAKE, FAKE, None, 0, FAKE, n3, None) == -1
    assert lib.adct_filter_save(FAKE, None, None, 0, FAKE, n1 - 1, None) == -5
