"""Pins of the inverse decoder for non-orthogonal matrices and of the coding
gain against the correlation (Sec. 2, 4.2.3, 4.3, 6.1.1)."""

import json
import os

import numpy as np
import pytest

from oracle import codec
from oracle import matrices as M
from oracle import nonortho as N
from synth import ar1_image

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NONORTHO = {"SDCT": M.t_sdct(), "BAS2008B": M.T_BAS2008B}


@pytest.mark.parametrize("name", ["SDCT", "BAS2008B", "T1", "LO"])
def test_adjugate_is_det_times_inverse(name):
    t = NONORTHO.get(name, M.TRANSFORMS.get(name))
    adj, det = N.adjugate_det(t)
    assert det == round(np.linalg.det(t.astype(np.float64)))
    assert np.allclose(adj / det, np.linalg.inv(t.astype(np.float64)), atol=1e-12)
    assert np.array_equal(t @ adj, det * np.eye(8, dtype=np.int64))


def test_the_two_competitors_are_not_orthogonal():
    for t in NONORTHO.values():
        g = t @ t.T
        assert np.count_nonzero(g - np.diag(np.diag(g))) > 0


@pytest.mark.parametrize("name", ["T1", "T2", "LO", "T6", "RDCT", "T4"])
def test_inverse_decoder_equals_transpose_decoder_for_orthogonal(name):
    # C_hat^-1 = C_hat^T when the rows are orthogonal
    img = ar1_image(48, 64, 0.95, seed=3)
    for r in (1, 5, 10, 37):
        a = N.evaluate(img, M.TRANSFORMS[name], r)
        b = codec.evaluate(img, M.TRANSFORMS[name], r)
        assert np.array_equal(a["rec"], b["rec"]) and a["sse"] == b["sse"]


@pytest.mark.parametrize("name", ["SDCT", "BAS2008B"])
def test_lossless_and_dc_only(name):
    t = NONORTHO[name]
    img = ar1_image(40, 56, 0.9, seed=4)
    assert N.evaluate(img, t, 64)["sse"] == 0
    # every row but the first sums to zero, so T^-1 e_0 = 1/8: r = 1 gives the
    # rounded block means
    assert np.all(t[1:].sum(axis=1) == 0)
    s = codec.to_blocks(img).sum(axis=(1, 2))
    want = codec.from_blocks(np.repeat(codec.rne_div(s, 64), 64).reshape(-1, 8, 8), 40, 56)
    assert np.array_equal(N.evaluate(img, t, 1)["rec"], want)


@pytest.mark.parametrize("name", ["SDCT", "BAS2008B"])
def test_inverse_decoder_against_float_inverse(name):
    # B = C_hat A C_hat^T, first r zig-zag kept, C_hat^-1 B' C_hat^-T in float64
    # with numpy's inverse: equal away from rounding ties
    t = NONORTHO[name]
    c = N.approx(t)
    ci = np.linalg.inv(c)
    img = ar1_image(64, 64, 0.95, seed=5)
    for r in (3, 10, 20):
        blocks = codec.to_blocks(img).astype(np.float64)
        b = np.einsum("ki,bij,lj->bkl", c, blocks, c)
        bk = codec.put_zigzag(codec.take_zigzag(b, r), r, np.float64)
        real = np.einsum("xk,bkl,yl->bxy", ci, bk, ci)
        rec = codec.from_blocks(np.clip(np.rint(real), 0, 255).astype(np.uint8), 64, 64)
        far = codec.from_blocks(np.abs(real - np.floor(real) - 0.5) > 1e-9, 64, 64)
        assert np.array_equal(N.evaluate(img, t, r)["rec"][far], rec[far])


def test_coding_gain_difference_at_the_table_correlation():
    rows = json.load(open(os.path.join(GOLD, "measures_table.json")))["rows"]
    mats = {"T1": M.T1, "LO": M.T_LO_X2, "T6": M.T6, "SDCT": M.t_sdct(), "BAS2008B": M.T_BAS2008B}
    for name, t in mats.items():
        d = float(N.cg_difference(N.approx(t), [0.95])[0])
        assert abs(d - (rows[name]["cg_star"] - rows["DCT"]["cg_star"])) < 2e-4, name


def test_coding_gain_difference_vanishes_without_correlation():
    # rho = 0: R_x = I and every orthonormal C_hat has C_g* = 0
    for t in (M.T1, M.T_LO_X2, M.T6, M.T_RDCT):
        assert abs(float(N.cg_difference(N.approx(t), [0.0])[0])) < 1e-12


def test_t1_has_the_smallest_loss_for_every_correlation():
    # Sec. 4.3: C_hat_1's coding-gain loss is below LO's and T6's for any rho,
    # and about half of LO's for highly correlated data
    rhos = np.linspace(0.02, 0.98, 49)
    d1 = N.cg_difference(N.approx(M.T1), rhos)
    dlo = N.cg_difference(N.approx(M.T_LO_X2), rhos)
    d6 = N.cg_difference(N.approx(M.T6), rhos)
    assert np.all(np.abs(d1) < np.abs(dlo)) and np.all(np.abs(d1) < np.abs(d6))
    ratio = abs(d1[-3]) / abs(dlo[-3])                      # rho = 0.94
    assert 0.3 < ratio < 0.7
