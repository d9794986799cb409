"""Pins of the SSIM oracle (Sec. 6.1.1's third figure of merit, defined by its
cited reference): the window, the valid-region filter against scipy, every map
entry against a direct per-window computation that uses centred moments, closed
forms for constant and shifted images, identity and symmetry."""

import math

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import ssim as S
from synth import ar1_image


def test_window():
    w = S.gaussian_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, :]) and np.allclose(w, w[:, ::-1])
    assert math.isclose(w[5, 6] / w[5, 5], math.exp(-1.0 / (2 * 1.5 ** 2)), rel_tol=1e-14)
    assert math.isclose(w[0, 0] / w[5, 5], math.exp(-50.0 / (2 * 1.5 ** 2)), rel_tol=1e-12)


def test_filter_matches_scipy():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (37, 29)).astype(np.float64)
    w = S.gaussian_window()
    np.testing.assert_allclose(S._filter_valid(img, w), correlate2d(img, w, mode="valid"), rtol=1e-13, atol=1e-10)


@pytest.fixture(scope="module")
def pair():
    x = ar1_image(48, 64, 0.9, seed=3).astype(np.int64)
    rng = np.random.default_rng(4)
    y = np.clip(x + rng.integers(-20, 21, x.shape), 0, 255)
    return x, y


def test_map_entries_by_direct_window(pair):
    x, y = pair
    m = S.ssim_map(x, y)
    assert m.shape == (38, 54)
    rng = np.random.default_rng(5)
    for i, j in zip(rng.integers(0, 38, 25), rng.integers(0, 54, 25)):
        assert math.isclose(m[i, j], S.ssim_window_brute(x, y, int(i), int(j)), rel_tol=1e-11, abs_tol=1e-12)


def test_identity_and_symmetry(pair):
    x, y = pair
    assert abs(S.ssim(x, x) - 1.0) < 1e-14
    assert math.isclose(S.ssim(x, y), S.ssim(y, x), rel_tol=1e-14)
    assert S.ssim(x, y) < 1.0


def test_constant_images():
    for a, b in [(0, 0), (100, 110), (0, 255), (37, 200)]:
        x = np.full((15, 20), a)
        y = np.full((15, 20), b)
        assert math.isclose(S.ssim(x, y), S.ssim_constant(a, b), rel_tol=1e-12)
    assert S.ssim_constant(0, 255) < 1e-3


def test_shift_keeps_structure_term():
    """y = x + c (no clipping): the local variances and the covariance are equal,
    so each window's SSIM reduces to its luminance term."""
    x = ar1_image(40, 40, 0.95, seed=6).astype(np.int64) // 2 + 40
    y = x + 25
    w = S.gaussian_window()
    m = S.ssim_map(x, y)
    mx = S._filter_valid(x.astype(np.float64), w)
    my = mx + 25.0
    np.testing.assert_allclose(m, (2 * mx * my + S.C1) / (mx * mx + my * my + S.C1), rtol=1e-9)


def test_too_small():
    with pytest.raises(ValueError):
        S.ssim(np.zeros((10, 40)), np.zeros((10, 40)))
