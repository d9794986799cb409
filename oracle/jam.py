"""16- and 32-point transforms by the Jridi-Alfalou-Meher construction (Sec. 6.2).

TEST INFRASTRUCTURE: see the package docstring.

From an N/2-point matrix T the construction builds the N-point matrix

    T_(N) = M_per diag(T, T) M_add          (the JAM recursion, Sec. 6.2)

where M_add = [[I, J], [J, -I]] (I identity, J counter-identity, both N/2 x N/2)
adds and subtracts the two halves of the input mirrored against each other, and
M_per is the perfect shuffle that puts output i of the upper copy of T at row 2i
and output i of the lower copy at row 2i + 1.  The factor 1/sqrt(2) of the
recursion is left out: it is merged into the scale S (Eq. (1)-(2)), which only
depends on the row norms.

Reading (the paper is not self-consistent here): the recursion as written
gives row 2i + 1 = [rev(t_i), -t_i], while the 16- and 32-point matrices the
paper prints have row 2i + 1 = [t_i, -rev(t_i)].  The two differ only in the
sign of the rows 2i + 1 with t_i antisymmetric (t_i = -rev(t_i)); a row sign
flips the sign of its coefficients and leaves the orthogonality, the scale and
every reconstruction unchanged (the quantiser rounds half away from zero, so
it is odd).  The printed matrices are the transform: `jam` builds them, and
`jam_as_written` builds the recursion literally, for the tests.

The N-point transform coder is the 8-point one with N x N blocks (`codec`):
zig-zag prefix of length r in [1, N^2], the optional quantiser, the transpose
inverse.  Reading for images whose sides are not multiples of N: the image is
extended to the next multiples of N by repeating its last row and column, coded,
and cropped back; the error counts the image's own pixels only.
"""

from __future__ import annotations

import numpy as np

from . import codec
from .matrices import row_norms2
from .sfg import OpCounter, t1_sfg


def jam(t: np.ndarray) -> np.ndarray:
    """One step of the construction in the sign convention of the printed
    matrices: row 2i = [t_i, rev(t_i)], row 2i + 1 = [t_i, -rev(t_i)]."""
    t = np.asarray(t)
    h = t.shape[0]
    out = np.zeros((2 * h, 2 * h), dtype=t.dtype)
    for i in range(h):
        out[2 * i, :h] = t[i]
        out[2 * i, h:] = t[i, ::-1]
        out[2 * i + 1, :h] = t[i]
        out[2 * i + 1, h:] = -t[i, ::-1]
    return out


def jam_as_written(t: np.ndarray) -> np.ndarray:
    """The recursion as a product of the three matrices of Sec. 6.2 (no 1/sqrt(2))."""
    t = np.asarray(t)
    h = t.shape[0]
    eye = np.eye(h, dtype=t.dtype)
    rev = eye[::-1]
    zero = np.zeros_like(t)
    m_add = np.block([[eye, rev], [rev, -eye]])
    blk = np.block([[t, zero], [zero, t]])
    m_per = np.zeros((2 * h, 2 * h), dtype=t.dtype)
    for i in range(h):
        m_per[2 * i, i] = 1
        m_per[2 * i + 1, h + i] = 1
    return m_per @ blk @ m_add


def jam_n(t8: np.ndarray, n: int) -> np.ndarray:
    """The n-point matrix (n in {8, 16, 32}) grown from an 8-point one."""
    t = np.asarray(t8, dtype=np.int64)
    while t.shape[0] < n:
        t = jam(t)
    if t.shape[0] != n:
        raise ValueError("n must be 8, 16 or 32")
    return t


def d_kron(n: int) -> np.ndarray:
    """diag(T_(n) T_(n)^T) for T1 in the Kronecker form the paper gives:
    D_(16) = 4 (I_2 x diag(4, 9, 10, 9) x I_2), D_(32) = 2 (D_(16) x I_2)."""
    i2 = np.eye(2, dtype=np.int64)
    d16 = 4 * np.kron(np.kron(i2, np.diag([4, 9, 10, 9])), i2)
    if n == 16:
        return np.diag(d16)
    if n == 32:
        return np.diag(2 * np.kron(d16, i2))
    raise ValueError("n must be 16 or 32")


def jam_fast(x, n: int, ops: OpCounter | None = None):
    """T1_(n) x by the recursion itself: n additions on the mirrored halves, then
    two n/2-point transforms, outputs interleaved; the 8-point core is the
    paper's signal-flow graph of T1 (Sec. 5.1).  Counts its operations in `ops`."""
    o = ops or OpCounter()
    x = list(x)
    if n == 8:
        return t1_sfg(x, o)
    h = n // 2
    up = [o.add(x[i], x[n - 1 - i]) for i in range(h)]        # x_top + rev(x_bottom)
    lo = [o.sub(x[i], x[n - 1 - i]) for i in range(h)]        # x_top - rev(x_bottom)
    yu, yl = jam_fast(up, h, o), jam_fast(lo, h, o)
    out = []
    for i in range(h):
        out += [yu[i], yl[i]]
    return out


def jam_cost(n: int) -> tuple[int, int]:
    """(additions, shifts) of one n-point T1_(n) transform by `jam_fast`."""
    o = OpCounter()
    jam_fast([0] * n, n, o)
    return o.adds, o.shifts


def pad_edge(img: np.ndarray, n: int) -> np.ndarray:
    """Extend the image to multiples of n by repeating its last row and column."""
    h, w = img.shape
    return np.pad(np.asarray(img), ((0, -h % n), (0, -w % n)), mode="edge")


def evaluate(img: np.ndarray, t_n: np.ndarray, r: int, step: int = 0) -> dict:
    """Code one image with the n-point matrix t_n (any H, W >= 1): the padded
    image goes through the transform coder of Sec. 6.1.1 with n x n blocks, the
    reconstruction is cropped back.  Returns rec, coef_int (blocks of the padded
    image in raster order, r levels each), sse, mse, psnr."""
    img = np.asarray(img, dtype=np.uint8)
    h, w = img.shape
    n = np.asarray(t_n).shape[0]
    if np.any(row_norms2(t_n) <= 0):
        raise ValueError("zero row")
    big = pad_edge(img, n)
    enc = codec.encode(big, t_n, r, step)
    dec = codec.decode(enc["coef_int"], t_n, r, big.shape[0], big.shape[1], step)
    rec = dec["rec"][:h, :w]
    s = codec.sse(img, rec)
    m = codec.mse_from_sse(s, h * w)
    return {"rec": rec, "coef_int": enc["coef_int"], "sse": s, "mse": m,
            "psnr": codec.psnr_from_mse(m)}
