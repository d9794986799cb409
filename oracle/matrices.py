"""Exact DCT, the paper's printed low-complexity matrices, and the scale S.

TEST INFRASTRUCTURE: see the package docstring.
"""

from __future__ import annotations

import math

import numpy as np

N = 8


def dct_matrix() -> np.ndarray:
    """Orthonormal 8-point DCT-II from its closed form (Sec. 2):
    C[k, n] = a_k cos((2n+1) k pi / 16), a_0 = 1/sqrt(8), a_k = 1/2.

    Reading: the matrix displayed in Sec. 2 (entries gamma_k = cos(2 pi (k+1)/32))
    is twice this one -- its first row is gamma_3 = 1/sqrt(2) instead of
    1/sqrt(8).  Only the orthonormal matrix reproduces the exact-DCT rows of
    the measures table of Sec. 4.3 (coding gain 8.8259 dB, efficiency 93.9912),
    so the orthonormal matrix is used everywhere."""
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    a = np.where(k == 0, 1.0 / math.sqrt(8.0), 0.5)
    return a * np.cos((2 * n + 1) * k * math.pi / (2 * N))


# The display of Sec. 2: entry = sign * gamma[index].
_PRINTED_IDX = [
    [3, 3, 3, 3, 3, 3, 3, 3],
    [0, 2, 4, 6, 6, 4, 2, 0],
    [1, 5, 5, 1, 1, 5, 5, 1],
    [2, 6, 0, 4, 4, 0, 6, 2],
    [3, 3, 3, 3, 3, 3, 3, 3],
    [4, 0, 6, 2, 2, 6, 0, 4],
    [5, 1, 1, 5, 5, 1, 1, 5],
    [6, 4, 2, 0, 0, 2, 4, 6],
]
_PRINTED_SGN = [
    [+1, +1, +1, +1, +1, +1, +1, +1],
    [+1, +1, +1, +1, -1, -1, -1, -1],
    [+1, +1, -1, -1, -1, -1, +1, +1],
    [+1, -1, -1, -1, +1, +1, +1, -1],
    [+1, -1, -1, +1, +1, -1, -1, +1],
    [+1, -1, +1, +1, -1, -1, +1, -1],
    [+1, -1, +1, -1, -1, +1, -1, +1],
    [+1, -1, +1, -1, +1, -1, +1, -1],
]


def dct_matrix_as_printed() -> np.ndarray:
    """The DCT matrix exactly as displayed in Sec. 2, gamma_k = cos(2 pi (k+1)/32)."""
    gamma = [math.cos(2.0 * math.pi * (k + 1) / 32.0) for k in range(7)]
    return np.array([[s * gamma[i] for i, s in zip(ri, rs)]
                     for ri, rs in zip(_PRINTED_IDX, _PRINTED_SGN)])


def _m(rows: str) -> np.ndarray:
    return np.array([[int(v) for v in r.split()] for r in rows.strip().splitlines()],
                    dtype=np.int64)


# New matrices found by the search over D2 (Sec. 4.1).
T1 = _m("""
1  1  1  1  1  1  1  1
2  2  1  0  0 -1 -2 -2
2  1 -1 -2 -2 -1  1  2
1  0 -2 -2  2  2  0 -1
1 -1 -1  1  1 -1 -1  1
2 -2  0  1 -1  0  2 -2
1 -2  2 -1 -1  2 -2  1
0 -1  2 -2  2 -2  1  0
""")

T2 = _m("""
1  1  1  1  1  1  1  1
2  1  2  0  0 -2 -1 -2
2  1 -1 -2 -2 -1  1  2
2  0 -2 -1  1  2  0 -2
1 -1 -1  1  1 -1 -1  1
1 -2  0  2 -2  0  2 -1
1 -2  2 -1 -1  2 -2  1
0 -2  1 -2  2 -1  2  0
""")

# Competitors, Sec. 2, table of common 8-point low-complexity matrices.
T_RDCT = _m("""
1  1  1  1  1  1  1  1
1  1  1  0  0 -1 -1 -1
1  0  0 -1 -1  0  0  1
1  0 -1 -1  1  1  0 -1
1 -1 -1  1  1 -1 -1  1
1 -1  0  1 -1  0  1 -1
0 -1  1  0  0  1 -1  0
0 -1  1 -1  1 -1  1  0
""")

T_BAS2008B = _m("""
1  1  1  1  1  1  1  1
1  1  1  0  0 -1 -1 -1
1  1 -1 -1 -1 -1  1  1
1  0 -1  0  0  1  0 -1
1 -1 -1  1  1 -1 -1  1
1 -1  1  0  0 -1  1 -1
1 -1  1 -1 -1  1 -1  1
1 -1  1 -1  1 -1  1 -1
""")

# T_LO has entries +-1/2; it is stored doubled so that it stays integral.
# S is invariant to a positive scaling of T, so S*T is unchanged.
T_LO_X2 = _m("""
2  2  2  2  2  2  2  2
2  2  2  0  0 -2 -2 -2
2  1 -1 -2 -2 -1  1  2
2  0 -2 -2  2  2  0 -2
2 -2 -2  2  2 -2 -2  2
2 -2  0  2 -2  0  2 -2
1 -2  2 -1 -1  2 -2  1
0 -2  2 -2  2 -2  2  0
""")

T6 = _m("""
1  1  1  1  1  1  1  1
2  1  1  0  0 -1 -1 -2
2  1 -1 -2 -2 -1  1  2
1  0 -2 -1  1  2  0 -1
1 -1 -1  1  1 -1 -1  1
1 -2  0  1 -1  0  2 -1
1 -2  2 -1 -1  2 -2  1
0 -1  1 -2  2 -1  1  0
""")

T4 = _m("""
1  1  1  1  1  1  1  1
1  1  1  0  0 -1 -1 -1
1  1 -1 -1 -1 -1  1  1
1  0 -1 -1  1  1  0 -1
1 -1 -1  1  1 -1 -1  1
1 -1  0  1 -1  0  1 -1
1 -1  1 -1 -1  1 -1  1
0 -1  1 -1  1 -1  1  0
""")


def t_sdct() -> np.ndarray:
    """Signed DCT: entry-wise signum of the DCT matrix (Sec. 2)."""
    return np.sign(dct_matrix()).astype(np.int64)


# Integer transforms the codec evaluates, by name.  "LO" is the doubled matrix.
TRANSFORMS = {
    "T1": T1,
    "T2": T2,
    "LO": T_LO_X2,
    "T6": T6,
    "RDCT": T_RDCT,
    "T4": T4,
}


def row_norms2(t: np.ndarray) -> np.ndarray:
    """diag(T T^T) as exact integers."""
    t = np.asarray(t, dtype=np.int64)
    return np.einsum("ij,ij->i", t, t)


def is_orthogonal_rows(t: np.ndarray) -> bool:
    """T T^T diagonal (Sec. 3.4): the rows form an orthogonal set."""
    g = np.asarray(t, dtype=np.int64) @ np.asarray(t, dtype=np.int64).T
    return bool(np.all(g == np.diag(np.diag(g))))


def scale_diag(t: np.ndarray) -> np.ndarray:
    """Diagonal of S in Eq. (2).

    Reading: S = diag(1/sqrt((T T^T)_kk)), i.e. each row of T normalised.
    For a T with orthogonal rows this equals the matrix square root of
    (T T^T)^-1 that Eq. (2) writes; for non-orthogonal T (BAS-2008b, SDCT) only
    the row-normalised form reproduces their rows of the measures table of
    Sec. 4.3 (the polar form does not)."""
    return 1.0 / np.sqrt(row_norms2(t).astype(np.float64))


def approx_matrix(t: np.ndarray) -> np.ndarray:
    """C_hat = S T, Eq. (1)."""
    return scale_diag(t)[:, None] * np.asarray(t, dtype=np.float64)


def polar_factor(t: np.ndarray) -> np.ndarray:
    """Orthogonal polar factor of T, (T T^T)^(-1/2) T, by eigendecomposition
    (the literal matrix-square-root form of Eq. (2))."""
    t = np.asarray(t, dtype=np.float64)
    w, v = np.linalg.eigh(t @ t.T)
    return (v * (1.0 / np.sqrt(w))) @ v.T @ t
