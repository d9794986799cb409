"""The paper's fast algorithm for T1 (Sec. 5.1) and its arithmetic cost.

TEST INFRASTRUCTURE: see the package docstring.

T1 = D A4 A3 A2 A1 with D = diag(1, 2, 1, 2, 1, 2, 1, 2): 24 additions and
6 multiplications by two, against 48 additions and 24 shifts for the direct
matrix product.  The signal-flow graph below merges D into A4 so that every
half in A4 cancels against a factor 2 of D.
"""

from __future__ import annotations

import numpy as np
from fractions import Fraction as F

H = F(1, 2)

# Factor matrices exactly as printed in Sec. 5.1 (blank entries are zero).
A1 = np.array([
    [1, 0, 0, 0, 0, 0, 0, 1],
    [0, 1, 0, 0, 0, 0, 1, 0],
    [0, 0, 1, 0, 0, 1, 0, 0],
    [0, 0, 0, 1, 1, 0, 0, 0],
    [0, 0, 0, 1, -1, 0, 0, 0],
    [0, 0, 1, 0, 0, -1, 0, 0],
    [0, 1, 0, 0, 0, 0, -1, 0],
    [1, 0, 0, 0, 0, 0, 0, -1],
], dtype=object)

A2 = np.array([
    [1, 0, 0, 1, 0, 0, 0, 0],
    [0, 1, 1, 0, 0, 0, 0, 0],
    [0, 1, -1, 0, 0, 0, 0, 0],
    [1, 0, 0, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 1, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, 0, 0],
    [0, 0, 0, 0, 0, 0, 1, 0],
    [0, 0, 0, 0, 0, 0, 0, 1],
], dtype=object)

A3 = np.array([
    [1, 1, 0, 0, 0, 0, 0, 0],
    [1, -1, 0, 0, 0, 0, 0, 0],
    [0, 0, 1, 0, 0, 0, 0, 0],
    [0, 0, 0, 1, 0, 0, 0, 0],
    [0, 0, 0, 0, 1, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, 0, 0],
    [0, 0, 0, 0, 0, 0, 1, 0],
    [0, 0, 0, 0, 0, 0, 0, 1],
], dtype=object)

A4 = np.array([
    [1, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, H, 1, 1],
    [0, 0, 1, 2, 0, 0, 0, 0],
    [0, 0, 0, 0, -1, -1, 0, H],
    [0, 1, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, H, 0, -1, 1],
    [0, 0, -2, 1, 0, 0, 0, 0],
    [0, 0, 0, 0, -1, 1, -H, 0],
], dtype=object)

D = np.diag(np.array([1, 2, 1, 2, 1, 2, 1, 2], dtype=object))


def factor_product() -> np.ndarray:
    """D A4 A3 A2 A1 in exact rational arithmetic."""
    return D.dot(A4).dot(A3).dot(A2).dot(A1)


class OpCounter:
    def __init__(self):
        self.adds = 0
        self.shifts = 0

    def add(self, a, b):
        self.adds += 1
        return a + b

    def sub(self, a, b):
        self.adds += 1
        return a - b

    def dbl(self, a):
        self.shifts += 1
        return a * 2


def t1_sfg(x, ops: OpCounter | None = None):
    """Forward T1 x by the signal-flow graph of the factorisation (stage by
    stage: A1 butterflies, A2 on the sum half, A3 on the first pair, then
    A4 with D folded in).  Works on numpy integer arrays elementwise."""
    o = ops or OpCounter()
    x0, x1, x2, x3, x4, x5, x6, x7 = x
    # A1
    a0, a1, a2, a3 = o.add(x0, x7), o.add(x1, x6), o.add(x2, x5), o.add(x3, x4)
    a4, a5, a6, a7 = o.sub(x3, x4), o.sub(x2, x5), o.sub(x1, x6), o.sub(x0, x7)
    # A2
    b0, b1, b2, b3 = o.add(a0, a3), o.add(a1, a2), o.sub(a1, a2), o.sub(a0, a3)
    # A3
    c0, c1 = o.add(b0, b1), o.sub(b0, b1)
    c2, c3, c4, c5, c6, c7 = b2, b3, a4, a5, a6, a7
    # D A4
    y0 = c0
    y1 = o.add(c5, o.dbl(o.add(c6, c7)))
    y2 = o.add(c2, o.dbl(c3))
    y3 = o.sub(c7, o.dbl(o.add(c4, c5)))
    y4 = c1
    y5 = o.add(c4, o.dbl(o.sub(c7, c6)))
    y6 = o.sub(c3, o.dbl(c2))
    y7 = o.sub(o.dbl(o.sub(c5, c4)), c6)
    return [y0, y1, y2, y3, y4, y5, y6, y7]


def sfg_cost() -> tuple[int, int]:
    """(additions, shifts) of one 8-point T1 transform by the SFG."""
    o = OpCounter()
    t1_sfg([0] * 8, o)
    return o.adds, o.shifts


def direct_cost(t: np.ndarray) -> tuple[int, int]:
    """(additions, shifts) of the direct product T x: per row, one addition
    fewer than its nonzero entries; one shift per entry of magnitude 2."""
    t = np.asarray(t, dtype=np.int64)
    adds = int(sum(max(int(np.count_nonzero(row)) - 1, 0) for row in t))
    shifts = int(np.count_nonzero(np.abs(t) == 2))
    return adds, shifts
