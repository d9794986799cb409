"""Pins of the oracle's transform-coding pipeline (Sec. 6.1.1)."""

import math
import os

import numpy as np
import pytest
from scipy.fft import dctn

from oracle import codec as Co
from oracle import matrices as M
from synth import ar1_image

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INT_T = ["T1", "T2", "LO", "T6", "RDCT", "T4"]


@pytest.fixture(scope="module")
def img():
    return ar1_image(64, 96, 0.95, seed=3)


def test_zigzag_is_jpeg():
    txt = open(os.path.join(GOLD, "jpeg_zigzag.txt")).read().split("\n")
    nat = [int(v) for line in txt if line and not line.startswith("#") for v in line.split()]
    assert [8 * i + j for i, j in Co.zigzag()] == nat


@pytest.mark.parametrize("r", [1, 3, 6, 10, 15, 21, 28, 36, 43, 49, 54, 58, 61, 63, 64])
def test_complete_antidiagonal_prefix_is_transpose_symmetric(r):
    m = Co.zonal_mask(r)
    assert np.array_equal(m, m.T)


def test_forward_int_is_two_sfg_passes(img):
    from oracle.sfg import t1_sfg
    blocks = Co.to_blocks(img)
    y = Co.forward_int(blocks, M.T1)
    # row pass then column pass with the flow graph (independent of the einsum)
    z = np.stack(t1_sfg([blocks[:, :, m] for m in range(8)]), axis=2)      # Z = A T^T
    y2 = np.stack(t1_sfg([z[:, x, :] for x in range(8)]), axis=1)          # Y = T Z
    assert np.array_equal(y, y2)


def test_dct_forward_matches_scipy(img):
    blocks = Co.to_blocks(img).astype(np.float64)
    b = Co.forward_real(blocks, M.dct_matrix())
    np.testing.assert_allclose(b, dctn(blocks, type=2, norm="ortho", axes=(1, 2)), atol=1e-10)


@pytest.mark.parametrize("name", INT_T)
def test_lossless_at_r64(img, name):
    res = Co.evaluate(img, M.TRANSFORMS[name], 64)
    assert res["sse"] == 0 and res["psnr"] == math.inf
    np.testing.assert_allclose(res["real"], img, atol=1e-9)


def test_dct_rational_coefficients_exact(img):
    """forward_dct equals scipy's orthonormal DCT-II everywhere, and its four
    rational coefficients equal the integer +-pixel sums over 8 exactly."""
    blocks = Co.to_blocks(img)
    b = Co.forward_dct(blocks)
    np.testing.assert_allclose(b, dctn(blocks.astype(np.float64), type=2, norm="ortho", axes=(1, 2)),
                               atol=1e-10)
    s4 = np.array([1, -1, -1, 1, 1, -1, -1, 1])
    a = blocks.astype(np.int64)
    assert np.array_equal(b[:, 0, 0] * 8, a.sum(axis=(1, 2)))
    assert np.array_equal(b[:, 4, 4] * 8, np.einsum("x,bxy,y->b", s4, a, s4))
    assert np.array_equal(b[:, 0, 4] * 8, np.einsum("bxy,y->b", a, s4))
    assert np.array_equal(b[:, 4, 0] * 8, np.einsum("x,bxy->b", s4, a))


def test_dct_quantiser_tie_rounds_away_from_zero():
    """A flat block of 3s has B(0,0) = 24 exactly; with step 16 that is 1.5
    steps, which the quantiser rounds away from zero to 2 (32), so r = 1
    reconstructs every pixel as 32 / 8 = 4."""
    img = np.full((8, 8), 3, dtype=np.uint8)
    res = Co.evaluate_dct(img, 1, 16)
    assert res["coef_scaled"][0, 0] == 24.0
    assert np.all(res["rec"] == 4)
    res = Co.evaluate_dct(np.full((8, 8), 1, dtype=np.uint8), 1, 16)       # 8 / 16 = 0.5 -> 1
    assert np.all(res["rec"] == 2)


def test_dct_lossless_at_r64(img):
    assert Co.evaluate_dct(img, 64)["sse"] == 0


@pytest.mark.parametrize("name", INT_T)
@pytest.mark.parametrize("r", [1, 5, 10, 33])
def test_parseval(img, name, r):
    # orthogonal C_hat: unrounded error energy = energy of the discarded coefficients
    t = M.TRANSFORMS[name]
    res = Co.evaluate(img, t, r)
    blocks = Co.to_blocks(img)
    b_all = Co.take_zigzag(Co.scale_coeffs(Co.forward_int(blocks, t), t), 64)
    discarded = float(np.sum(b_all[:, r:] ** 2))
    assert abs(res["mse_real"] * img.size - discarded) <= 1e-9 * max(discarded, 1.0)


@pytest.mark.parametrize("name", INT_T)
def test_exact_inverse_matches_float(img, name):
    t = M.TRANSFORMS[name]
    enc = Co.encode(img, t, 10)
    y_full = Co.put_zigzag(enc["coef_int"], 10, np.int64)
    num, big_l = Co.inverse_exact(y_full, t)
    b_full = Co.put_zigzag(enc["coef_scaled"], 10, np.float64)
    real = Co.inverse_real(b_full, M.approx_matrix(t))
    np.testing.assert_allclose(num / big_l, real, atol=1e-9)


@pytest.mark.parametrize("name", INT_T)
def test_level_shift_invariance(img, name):
    t = M.TRANSFORMS[name]
    shifted = img.astype(np.int64) - 128
    res = Co.evaluate(img, t, 10)
    enc = Co.encode(img, t, 10)
    blocks = Co.to_blocks(shifted)
    y = Co.take_zigzag(Co.forward_int(blocks, t), 10)
    assert np.array_equal(y[:, 1:], enc["coef_int"][:, 1:])   # only DC moves
    y_full = Co.put_zigzag(y, 10, np.int64)
    num, big_l = Co.inverse_exact(y_full, t)
    rec = Co.from_blocks(np.clip(Co.rne_div(num, big_l) + 128, 0, 255), *img.shape)
    assert np.array_equal(rec, res["rec"])


def test_r1_is_rounded_block_mean(img):
    # r = 1 keeps only DC: the block is replaced by its mean (all DC rows are flat)
    blocks = Co.to_blocks(img)
    s = blocks.sum(axis=(1, 2))
    mean_rne = np.array([int(round(v / 64)) if (v % 64) * 2 != 64 else
                         (v // 64 if (v // 64) % 2 == 0 else v // 64 + 1) for v in s])
    ref = Co.from_blocks(np.repeat(mean_rne, 64).reshape(-1, 8, 8), *img.shape)
    for name in INT_T:
        assert np.array_equal(Co.evaluate(img, M.TRANSFORMS[name], 1)["rec"], ref)


def test_rne_div():
    num = np.arange(-1000, 1000)
    got = Co.rne_div(num, 8)
    ref = np.array([round(v / 8) for v in num])          # Python rounds half to even
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["T1", "T6", "RDCT"])
def test_quantizer_exhaustive(name):
    # q = round-half-away(Y s_k s_l / 16) for every |Y| <= 18360 and every scale
    # class, against an exact integer restatement: q = k iff
    # (2k-1)^2 * 256 m <= 4 Y^2 < (2k+1)^2 * 256 m  with m = n_k n_l (k >= 1).
    t = M.TRANSFORMS[name]
    n = M.row_norms2(t)
    y = np.arange(-18360, 18361, dtype=np.int64)
    zi, zj = Co.zz_index_arrays()
    step = 16
    seen = set()
    for p in range(64):
        m = int(n[zi[p]] * n[zj[p]])
        if m in seen:
            continue
        seen.add(m)
        ycols = np.repeat(y[:, None], p + 1, axis=1)
        q = Co.quantize(ycols, t, p + 1, step)[:, p]
        a = np.abs(q)
        four_y2 = 4 * y * y
        ok_hi = four_y2 < (2 * a + 1) ** 2 * step * step * m
        ok_lo = (a == 0) | (four_y2 >= (2 * a - 1) ** 2 * step * step * m)
        assert np.all(ok_hi & ok_lo), (name, m)
        assert np.all(np.sign(q) == np.sign(y) * (a > 0))


def test_quantized_roundtrip_bounds(img):
    # dequantisation error per coefficient is at most step/2 in the orthonormal domain
    t = M.T1
    res = Co.evaluate(img, t, 10, step=16)
    enc = Co.encode(img, t, 10, step=16)
    assert np.all(np.abs(enc["coef_scaled"] - 16 * enc["coef_int"]) <= 8 + 1e-9)
    assert res["psnr"] < Co.evaluate(img, t, 10)["psnr"] + 1e-9


def test_t1_beats_lo_and_t6_on_ar1():
    # Sec. 6.1.1 reports C_hat_1 above C_hat_LO and C_hat_6 in PSNR for every r
    img = ar1_image(256, 256, 0.95, seed=0)
    for r in (3, 10, 20):
        p1 = Co.evaluate(img, M.T1, r)["psnr"]
        assert p1 > Co.evaluate(img, M.T_LO_X2, r)["psnr"]
        assert p1 > Co.evaluate(img, M.T6, r)["psnr"]
