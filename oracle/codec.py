"""Blockwise 8x8 transform coding, written out from its definition (Sec. 6.1.1).

TEST INFRASTRUCTURE: see the package docstring.

The same steps serve the 16- and 32-point matrices of the JAM construction
(Sec. 6.2; see `jam`): the block order is the order of T.

Per 8x8 block A of an 8-bit image:
  forward   B = C_hat A C_hat^T with C_hat = S T           (Sec. 6.1.1, Eq. (1))
            computed as the exact integer stage Y = T A T^T, then B = S Y S
  retain    the first r coefficients of the zig-zag scan, the rest set to 0
  inverse   A_rec = C_hat^T B' C_hat  (orthogonal T only)  (Sec. 6.1.1)
  score     MSE and PSNR of the rounded, clipped reconstruction

Readings (the paper is silent on these):
  * no level shift of the pixels before the transform;
  * the zig-zag scan is the JPEG one (row index = vertical frequency);
  * the reconstruction is rounded half-to-even and clipped to [0, 255] before
    the error is measured, since the compared images are 8-bit;
  * PSNR = 10 log10(255^2 / MSE), MSE = SSE / (H W);
  * the optional quantiser (not in the paper) is q = round-half-away(B / step),
    dequantised as step*q.
"""

from __future__ import annotations

import math
from functools import reduce

import numpy as np

from .matrices import approx_matrix, dct_matrix, is_orthogonal_rows, row_norms2, scale_diag

N = 8


# --------------------------------------------------------------------------
# zig-zag
# --------------------------------------------------------------------------

def zigzag(n: int = N) -> list[tuple[int, int]]:
    """JPEG zig-zag order of an n x n block as (i, j) = (row, column).

    Anti-diagonals d = i + j are visited in increasing order; on odd d the row
    index increases along the diagonal, on even d it decreases."""
    out = []
    for d in range(2 * n - 1):
        lo, hi = max(0, d - n + 1), min(d, n - 1)
        rows = range(lo, hi + 1) if d % 2 == 1 else range(hi, lo - 1, -1)
        out.extend((i, d - i) for i in rows)
    return out


def zonal_mask(r: int, n: int = N) -> np.ndarray:
    """Boolean n x n mask of the first r zig-zag coefficients (Sec. 6.1.1)."""
    if not 0 <= r <= n * n:
        raise ValueError(f"r must be in [0, {n * n}]")
    m = np.zeros((n, n), dtype=bool)
    for i, j in zigzag(n)[:r]:
        m[i, j] = True
    return m


def zz_index_arrays(n: int = N) -> tuple[np.ndarray, np.ndarray]:
    zz = zigzag(n)
    return np.array([p[0] for p in zz]), np.array([p[1] for p in zz])


# --------------------------------------------------------------------------
# blocks
# --------------------------------------------------------------------------

def to_blocks(img: np.ndarray, n: int = N) -> np.ndarray:
    """(H, W) image -> (H/n * W/n, n, n) blocks in raster order, int64."""
    h, w = img.shape
    if h % n or w % n:
        raise ValueError(f"H and W must be multiples of {n}")
    b = np.asarray(img, dtype=np.int64).reshape(h // n, n, w // n, n)
    return b.transpose(0, 2, 1, 3).reshape(-1, n, n)


def from_blocks(blocks: np.ndarray, h: int, w: int, n: int = N) -> np.ndarray:
    b = np.asarray(blocks).reshape(h // n, w // n, n, n).transpose(0, 2, 1, 3)
    return b.reshape(h, w)


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------

def forward_int(blocks: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Exact integer stage Y = T A T^T for every block (int64)."""
    t = np.asarray(t, dtype=np.int64)
    return np.einsum("ki,bij,lj->bkl", t, np.asarray(blocks, dtype=np.int64), t,
                     optimize=True)


def scale_coeffs(y: np.ndarray, t: np.ndarray) -> np.ndarray:
    """B = S Y S, i.e. B_kl = s_k s_l Y_kl (Eq. (1) applied on both sides)."""
    s = scale_diag(t)
    return np.asarray(y, dtype=np.float64) * (s[:, None] * s[None, :])


def forward_real(blocks: np.ndarray, c: np.ndarray) -> np.ndarray:
    """B = C A C^T for a real matrix C (used for the exact DCT), float64."""
    return np.einsum("ki,bij,lj->bkl", c, np.asarray(blocks, dtype=np.float64), c,
                     optimize=True)


def take_zigzag(coef: np.ndarray, r: int) -> np.ndarray:
    """(nb, n, n) -> (nb, r) in zig-zag order."""
    zi, zj = zz_index_arrays(coef.shape[-1])
    return coef[:, zi[:r], zj[:r]]


def put_zigzag(vals: np.ndarray, r: int, dtype, n: int = N) -> np.ndarray:
    """(nb, r) zig-zag prefix -> (nb, n, n) with the discarded entries 0."""
    zi, zj = zz_index_arrays(n)
    out = np.zeros((vals.shape[0], n, n), dtype=dtype)
    out[:, zi[:r], zj[:r]] = vals
    return out


# --------------------------------------------------------------------------
# quantiser (not in the paper)
# --------------------------------------------------------------------------

def _round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def quantize(y_zz: np.ndarray, t: np.ndarray, r: int, step: int) -> np.ndarray:
    """q = round-half-away(B / step) for the retained coefficients, B = s_k s_l Y.

    Reading: where n_k n_l = (T T^T)_kk (T T^T)_ll is a perfect square m^2 the
    quotient B/step = Y/(step m) is rational and can sit exactly on a half, so
    it is rounded in exact integer arithmetic; otherwise it is irrational
    (never an exact half) and float64 decides."""
    n = row_norms2(t)
    zi, zj = zz_index_arrays(np.asarray(t).shape[0])
    y_zz = np.asarray(y_zz, dtype=np.int64)
    q = np.empty_like(y_zz)
    s = scale_diag(t)
    for p in range(r):
        k, l = zi[p], zj[p]
        prod = int(n[k] * n[l])
        m = math.isqrt(prod)
        col = y_zz[:, p]
        if m * m == prod:
            d = step * m
            q[:, p] = np.sign(col) * ((2 * np.abs(col) + d) // (2 * d))
        else:
            b = col.astype(np.float64) * (s[k] * s[l])
            q[:, p] = _round_half_away(b / step).astype(np.int64)
    return q


# --------------------------------------------------------------------------
# inverse
# --------------------------------------------------------------------------

def _lcm(vals) -> int:
    return reduce(lambda a, b: a * b // math.gcd(a, b), (int(v) for v in vals), 1)


def rne_div(num: np.ndarray, den: int) -> np.ndarray:
    """Exact round-half-to-even of num/den for int64 num and positive int den."""
    q, rem = np.divmod(np.asarray(num, dtype=np.int64), den)   # floor division
    twice = 2 * rem
    up = (twice > den) | ((twice == den) & (q % 2 == 1))
    return q + up.astype(np.int64)


def inverse_exact(y_full: np.ndarray, t: np.ndarray):
    """A_rec = C_hat^T (S Y' S) C_hat = T^T (Y' o W) T with W_kl = 1/(n_k n_l),
    computed exactly: returns (numerator, L) with A_rec = numerator / L,
    L = lcm over (k, l) of n_k n_l.  Y' is the integer stage with discarded
    coefficients already zeroed.  Only valid for T with orthogonal rows."""
    t = np.asarray(t, dtype=np.int64)
    if not is_orthogonal_rows(t):
        raise ValueError("the transpose inverse needs T T^T diagonal (Sec. 6.1.1)")
    n = row_norms2(t)
    nn = n[:, None] * n[None, :]
    big_l = _lcm(nn.ravel())
    w = big_l // nn
    num = np.einsum("ki,bkl,lj->bij", t, np.asarray(y_full, dtype=np.int64) * w, t,
                    optimize=True)
    return num, big_l


def inverse_real(b_full: np.ndarray, c_hat: np.ndarray) -> np.ndarray:
    """A_rec = C_hat^T B' C_hat in float64 (Sec. 6.1.1)."""
    return np.einsum("ki,bkl,lj->bij", c_hat, np.asarray(b_full, dtype=np.float64), c_hat,
                     optimize=True)


def _settle_near_halves(rounded, real, q_zz, t, r, step, window=1e-6):
    """Round-half-to-even of the EXACT dequantised reconstruction where float64
    is too close to a half to decide.

    A_rec(x, y) = sum_kl T[k, x] T[l, y] step q_kl / sqrt(n_k n_l) is a sum of
    square roots; at pixels whose float64 value lies within `window` of a half
    it is recomputed with 60 significant digits.  A value within 1e-40 of a
    half is an exact half (a nonzero distance for these bounded integer
    combinations is many orders of magnitude larger), rounded to even."""
    from decimal import Decimal, localcontext
    frac = np.abs(real - np.floor(real) - 0.5)
    idx = np.argwhere(frac < window)
    if idx.size == 0:
        return
    t = np.asarray(t, dtype=np.int64)
    n = row_norms2(t)
    zz = zigzag(t.shape[0])[:r]
    with localcontext() as ctx:
        ctx.prec = 60
        inv_sqrt = {(k, l): 1 / Decimal(int(n[k] * n[l])).sqrt() for k, l in zz}
        half = Decimal(1) / 2
        for b, x, y in idx:
            acc = Decimal(0)
            for p, (k, l) in enumerate(zz):
                c = int(t[k, x] * t[l, y] * step * q_zz[b, p])
                if c:
                    acc += c * inv_sqrt[(k, l)]
            fl = acc.to_integral_value(rounding="ROUND_FLOOR")
            d = acc - fl - half
            if abs(d) < Decimal("1e-40"):
                v = fl if int(fl) % 2 == 0 else fl + 1
            else:
                v = fl + 1 if d > 0 else fl
            rounded[b, x, y] = float(v)


def clip_u8(x: np.ndarray) -> np.ndarray:
    return np.clip(x, 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# scores
# --------------------------------------------------------------------------

def sse(a: np.ndarray, b: np.ndarray) -> int:
    d = np.asarray(a, dtype=np.int64) - np.asarray(b, dtype=np.int64)
    return int(np.sum(d * d))


def mse_from_sse(s: float, npix: int) -> float:
    return float(s) / float(npix)


def psnr_from_mse(m: float) -> float:
    """PSNR = 10 log10(255^2 / MSE); +inf when MSE == 0."""
    return math.inf if m == 0 else 10.0 * math.log10(255.0 * 255.0 / m)


# --------------------------------------------------------------------------
# whole pipeline
# --------------------------------------------------------------------------

def encode(img: np.ndarray, t: np.ndarray, r: int, step: int = 0) -> dict:
    """Forward transform of every block; first r zig-zag coefficients.

    Returns coef_int (nb, r): the exact integer stage Y (or, with step > 0, the
    quantised q), and coef_scaled (nb, r): B = s_k s_l Y in float64.  The block
    size n is the order of T (8, or 16 and 32 for the JAM matrices)."""
    n = np.asarray(t).shape[0]
    if not 1 <= r <= n * n:
        raise ValueError(f"r must be in [1, {n * n}]")
    blocks = to_blocks(img, n)
    y = forward_int(blocks, t)
    y_zz = take_zigzag(y, r)
    b_zz = take_zigzag(scale_coeffs(y, t), r)
    out = {"coef_scaled": b_zz, "y": y_zz}
    out["coef_int"] = quantize(y_zz, t, r, step) if step > 0 else y_zz
    return out


def decode(coef_int: np.ndarray, t: np.ndarray, r: int, h: int, w: int,
           step: int = 0) -> dict:
    """Inverse of `encode`'s integer output.  Returns the rounded, clipped uint8
    image `rec` and the real-valued reconstruction `real` (float64)."""
    n = np.asarray(t).shape[0]
    if step == 0:
        y_full = put_zigzag(coef_int, r, np.int64, n)
        num, big_l = inverse_exact(y_full, t)
        rounded = rne_div(num, big_l)
        real = num.astype(np.float64) / big_l
    else:
        bq = put_zigzag(np.asarray(coef_int, dtype=np.float64) * step, r, np.float64, n)
        real = inverse_real(bq, approx_matrix(t))
        rounded = np.rint(real)
        _settle_near_halves(rounded, real, np.asarray(coef_int, dtype=np.int64), t, r, step)
    return {"rec": from_blocks(clip_u8(rounded), h, w, n),
            "real": from_blocks(real, h, w, n)}


def evaluate(img: np.ndarray, t: np.ndarray, r: int, step: int = 0) -> dict:
    """Encode, decode and score one image with integer transform T."""
    h, w = img.shape
    enc = encode(img, t, r, step)
    dec = decode(enc["coef_int"], t, r, h, w, step)
    s = sse(img, dec["rec"])
    m = mse_from_sse(s, h * w)
    d = np.asarray(img, dtype=np.float64) - dec["real"]
    return {**enc, **dec, "sse": s, "mse": m, "psnr": psnr_from_mse(m),
            "mse_real": float(np.mean(d * d))}


def forward_dct(blocks: np.ndarray) -> np.ndarray:
    """B = C A C^T with the orthonormal DCT (Sec. 2) in float64, except the four
    coefficients (k, l) in {0, 4}^2, which are rational and computed exactly.

    a_0 = 1/sqrt(8) and a_4 cos((2n+1) 4 pi / 16) = +-1/sqrt(8), so every basis
    entry of those four is +-1/8 and B(k, l) = (sum of +-pixels) / 8 exactly.
    The quantiser's half-step cases land on them (B(0,0)/16 is a half for one
    8-bit block in 128); float64 would decide such a tie by its own rounding
    of 1/sqrt(8)^2."""
    b = forward_real(blocks, dct_matrix())
    a = np.asarray(blocks, dtype=np.int64)
    sign = {0: np.ones(N, dtype=np.int64), 4: np.array([1, -1, -1, 1, 1, -1, -1, 1], dtype=np.int64)}
    for k in (0, 4):
        for l in (0, 4):
            b[:, k, l] = np.einsum("x,bxy,y->b", sign[k], a, sign[l]) / 8.0
    return b


def evaluate_dct(img: np.ndarray, r: int, step: int = 0) -> dict:
    """The same pipeline with the exact (orthonormal) DCT in float64."""
    h, w = img.shape
    c = dct_matrix()
    blocks = to_blocks(img)
    b = forward_dct(blocks)
    b_zz = take_zigzag(b, r)
    if step > 0:
        b_zz_kept = _round_half_away(b_zz / step) * step
    else:
        b_zz_kept = b_zz
    real = inverse_real(put_zigzag(b_zz_kept, r, np.float64), c)
    rec = from_blocks(clip_u8(np.rint(real)), h, w)
    s = sse(img, rec)
    m = mse_from_sse(s, h * w)
    return {"coef_scaled": b_zz, "rec": rec, "real": from_blocks(real, h, w),
            "sse": s, "mse": m, "psnr": psnr_from_mse(m)}
