"""Non-orthogonal low-complexity matrices in the transform coder, and the
coding gain against the inter-pixel correlation (Sec. 2, Sec. 4.2.3, Sec. 6.1.1).

TEST INFRASTRUCTURE: see the package docstring.

The signed DCT (T = sgn(C)) and BAS-2008b are the paper's non-orthogonal
competitors.  With C_hat = S T (S = diag(1/sqrt(diag(T T^T))), reading of Eq. (2)
used throughout) the transpose is not the inverse; Sec. 6.1.1 states the transpose
inverse for orthogonal approximations only, and the general decoder is

    A_rec = C_hat^-1 B' C_hat^-T.

Zonal coding only (the paper's image experiment): B' keeps the first r zig-zag
coefficients of B = C_hat A C_hat^T = S Y S with Y = T A T^T, so
A_rec = T^-1 S^-1 (S Y' S) S^-1 T^-T = T^-1 Y' T^-T exactly, a rational number:
with T^-1 = adj(T) / det(T) it is adj(T) Y' adj(T)^T / det(T)^2, computed here in
exact integer arithmetic and rounded half to even.

The coding-gain curve of Sec. 4.3 (difference of the unified coding gain of an
approximation and of the exact DCT for 0 < rho < 1) is `cg_difference`.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import codec
from .matrices import dct_matrix
from .measures import unified_coding_gain


def adjugate_det(t: np.ndarray) -> tuple[np.ndarray, int]:
    """(adj(T), det(T)) of an integer matrix by exact Gauss-Jordan elimination
    over the rationals: adj(T) = det(T) T^-1."""
    n = t.shape[0]
    a = [[Fraction(int(v)) for v in row] + [Fraction(int(i == j)) for j in range(n)]
         for i, row in enumerate(np.asarray(t))]
    det = Fraction(1)
    for c in range(n):
        piv = next((r for r in range(c, n) if a[r][c] != 0), None)
        if piv is None:
            raise ValueError("singular matrix")
        if piv != c:
            a[c], a[piv] = a[piv], a[c]
            det = -det
        p = a[c][c]
        det *= p
        a[c] = [v / p for v in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c]
                a[r] = [x - f * y for x, y in zip(a[r], a[c])]
    inv = [row[n:] for row in a]
    adj = np.array([[int(v * det) for v in row] for row in inv], dtype=object)
    assert all((v * det).denominator == 1 for row in inv for v in row)
    return adj.astype(np.int64), int(det)


def evaluate(img: np.ndarray, t: np.ndarray, r: int) -> dict:
    """Zonal coding of one image (H, W multiples of 8) with an invertible integer
    T and the inverse decoder.  Returns rec, sse, mse, psnr."""
    img = np.asarray(img, dtype=np.uint8)
    h, w = img.shape
    if not 1 <= r <= 64:
        raise ValueError("r must be in [1, 64]")
    t = np.asarray(t, dtype=np.int64)
    adj, det = adjugate_det(t)
    blocks = codec.to_blocks(img)
    y = codec.forward_int(blocks, t)
    y_kept = codec.put_zigzag(codec.take_zigzag(y, r), r, np.int64)
    num = np.einsum("xk,bkl,yl->bxy", adj, y_kept, adj, optimize=True)   # adj Y' adj^T
    rec_blocks = np.clip(codec.rne_div(num, det * det), 0, 255).astype(np.uint8)
    rec = codec.from_blocks(rec_blocks, h, w)
    s = codec.sse(img, rec)
    m = codec.mse_from_sse(s, h * w)
    return {"rec": rec, "sse": s, "mse": m, "psnr": codec.psnr_from_mse(m)}


def approx(t: np.ndarray) -> np.ndarray:
    """C_hat = S T with S = diag(1 / sqrt(diag(T T^T)))."""
    t = np.asarray(t, dtype=np.float64)
    return t / np.sqrt(np.sum(t * t, axis=1))[:, None]


def cg_difference(c_hat: np.ndarray, rhos) -> np.ndarray:
    """C_g*(C_hat, rho) - C_g*(C, rho) over the given correlations (the curve of
    Sec. 4.3's coding-gain figure, in dB; negative: C_hat compacts less)."""
    c = dct_matrix()
    return np.array([unified_coding_gain(c_hat, float(p)) - unified_coding_gain(c, float(p))
                     for p in rhos])
