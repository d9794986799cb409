"""Structural similarity (SSIM) of a reconstruction, the third figure of merit of
Sec. 6.1.1 (TEST INFRASTRUCTURE: see the package docstring).

The paper names SSIM and cites its original definition without restating it.
Reading (the definition of that reference, as its authors specified it):
  * local statistics over an 11 x 11 circularly-symmetric Gaussian window,
    standard deviation 1.5 pixels, normalised to unit sum;
  * SSIM(x, y) = (2 mu_x mu_y + C1)(2 s_xy + C2) /
                 ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
    C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = 255, with the weighted means mu,
    variances s^2 = E_w[x^2] - mu^2 and covariance s_xy = E_w[xy] - mu_x mu_y;
  * the map is evaluated where the window lies inside the image (no padding),
    and the image's SSIM is the mean of the map; no downsampling.
Everything is float64.
"""

from __future__ import annotations

import math

import numpy as np

WIN = 11
SIGMA = 1.5
K1, K2, L = 0.01, 0.03, 255.0
C1 = (K1 * L) ** 2
C2 = (K2 * L) ** 2


def gaussian_window() -> np.ndarray:
    """11 x 11 Gaussian weights exp(-(dx^2 + dy^2) / (2 sigma^2)), unit sum."""
    r = np.arange(WIN) - (WIN - 1) / 2.0
    w = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * SIGMA ** 2))
    return w / w.sum()


def _filter_valid(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum over the window of w * img at every position where it fits (no padding):
    out[i, j] = sum_{a, b} w[a, b] img[i + a, j + b]."""
    h, wd = img.shape
    oh, ow = h - WIN + 1, wd - WIN + 1
    out = np.zeros((oh, ow))
    for a in range(WIN):
        for b in range(WIN):
            out += w[a, b] * img[a:a + oh, b:b + ow]
    return out


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM at every window position inside the image."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape or x.ndim != 2 or min(x.shape) < WIN:
        raise ValueError("two equal 2-D images of at least 11 x 11 are required")
    w = gaussian_window()
    mx, my = _filter_valid(x, w), _filter_valid(y, w)
    sxx = _filter_valid(x * x, w) - mx * mx
    syy = _filter_valid(y * y, w) - my * my
    sxy = _filter_valid(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim(x: np.ndarray, y: np.ndarray) -> float:
    """Mean SSIM of y against x."""
    return float(np.mean(ssim_map(x, y)))


def ssim_constant(a: float, b: float) -> float:
    """Closed form for two constant images a and b (all local variances vanish)."""
    return (2 * a * b + C1) / (a * a + b * b + C1)


def ssim_window_brute(x: np.ndarray, y: np.ndarray, i: int, j: int) -> float:
    """SSIM of the single window whose top-left pixel is (i, j), by direct sums."""
    w = gaussian_window()
    xs = np.asarray(x, dtype=np.float64)[i:i + WIN, j:j + WIN]
    ys = np.asarray(y, dtype=np.float64)[i:i + WIN, j:j + WIN]
    mx = float(np.sum(w * xs))
    my = float(np.sum(w * ys))
    vx = float(np.sum(w * (xs - mx) ** 2))
    vy = float(np.sum(w * (ys - my) ** 2))
    cxy = float(np.sum(w * (xs - mx) * (ys - my)))
    return ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))


def mean_ssim_table(images, recons) -> np.ndarray:
    """SSIM of each reconstruction against its image."""
    return np.array([ssim(a, b) for a, b in zip(images, recons)])


__all__ = ["WIN", "SIGMA", "C1", "C2", "gaussian_window", "ssim_map", "ssim", "ssim_constant",
           "ssim_window_brute", "mean_ssim_table"]
assert math.isclose(C1, 6.5025) and math.isclose(C2, 58.5225)
