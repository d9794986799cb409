"""Rate-distortion sweep over a set of images (Sec. 6.1.1).

TEST INFRASTRUCTURE: see the package docstring.

The paper evaluates every transform on every image for each retained count r
and averages MSE / PSNR over the images (Sec. 6.1.1).  The sweep here is that
definition written as a plain loop: one full encode / decode / score per
(image, transform, r), no incremental reuse.
"""

from __future__ import annotations

import numpy as np

from . import codec as Co
from . import matrices as M


def sse_table(images, transforms, r_lo: int = 1, r_hi: int = 63) -> np.ndarray:
    """uint64 [n_images][n_transforms][r_hi - r_lo + 1] of squared errors of the
    rounded, clipped reconstruction.  Transform names: "DCT" (float64, exact
    DCT) or a key of matrices.TRANSFORMS (exact integer arithmetic)."""
    out = np.zeros((len(images), len(transforms), r_hi - r_lo + 1), dtype=np.uint64)
    for i, img in enumerate(images):
        for t, name in enumerate(transforms):
            for r in range(r_lo, r_hi + 1):
                if name == "DCT":
                    res = Co.evaluate_dct(img, r)
                else:
                    res = Co.evaluate(img, M.TRANSFORMS[name], r)
                out[i, t, r - r_lo] = res["sse"]
    return out


def mean_psnr(table: np.ndarray, sizes) -> np.ndarray:
    """Average PSNR over images for each (transform, r), as in the curves of
    Sec. 6.1.1 (mean of per-image PSNR values)."""
    npix = np.array([h * w for h, w in sizes], dtype=np.float64)
    with np.errstate(divide="ignore"):
        psnr = 10.0 * np.log10(255.0 * 255.0 * npix[:, None, None] / table.astype(np.float64))
    return psnr.mean(axis=0)
