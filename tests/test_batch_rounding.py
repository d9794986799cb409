"""The integer rate-distortion sweep rounds its exact reconstruction numerators
n / L (L = lcm(n_k)^2, Sec. 6.1.1 inverse over the orthogonal rows of Sec. 3.4)
to the nearest integer, ties to even, clipped to [0, 255], through one float32
fma: with P = n + L/2 and L = 2^s d, q = trunc(fma(P >> s, 1/d, 1/(2d))), the
remainder P - L q flags a tie, and a saturating byte pack clips.  This test
emulates that float32 arithmetic bit for bit in integers and compares it with
exact rounding for every numerator in [-2L, 258L] (the range where the clip
does not decide the result) and with random numerators over the whole range
the sweep can reach (|n| <= 2040 L), for all six integer transforms."""

import math

import numpy as np
import pytest

from oracle import matrices as M

NAMES = ["T1", "T2", "LO", "T6", "RDCT", "T4"]


def _params(name):
    t = np.array(M.TRANSFORMS[name], dtype=np.int64)
    lcm = 1
    for v in np.diag(t @ t.T):
        lcm = lcm * int(v) // math.gcd(lcm, int(v))
    L = lcm * lcm
    s = 0
    if L >= 4096:
        while (L >> s) & 1 == 0:
            s += 1
    return L, s, L >> s


def _f32_parts(x: float):
    """x = m * 2^e with m a 24-bit integer, for a positive normal float32."""
    f = np.float32(x)
    mant, exp = np.frexp(np.float64(f))          # f = mant * 2^exp, 0.5 <= mant < 1
    m = int(mant * (1 << 24))
    assert float(m) == mant * (1 << 24)
    return m, int(exp) - 24


def _kernel_q(P, L, s, d, tie_fix=True):
    """The kernel's rne_int followed by the saturating pack, emulated exactly."""
    inv = np.float32(1.0) / np.float32(d)
    off = np.float32(0.5) / np.float32(d)
    m, e = _f32_parts(float(inv))
    m2, e2 = _f32_parts(float(off))
    assert m2 == m and e2 == e - 1                # the offset is exactly half of 1/d
    v = P >> s                                    # arithmetic shift, as on the device
    # fma(v, inv, off) = m (2v + 1) 2^(e-1) exactly; round to 24 bits, ties to even
    N = m * (2 * v + 1)
    a = np.abs(N)
    bl = np.frexp(a.astype(np.float64))[1]        # bit length (a < 2^53)
    sh = np.maximum(bl - 24, 0)
    lo = a & ((np.int64(1) << sh) - 1)
    half = np.where(sh > 0, np.int64(1) << np.maximum(sh - 1, 0), 0)
    r = a >> sh
    up = (sh > 0) & ((lo > half) | ((lo == half) & ((r & 1) == 1)))
    r = (r + up) << sh                            # |rounded| as an integer times 2^(e-1)
    q = np.sign(N) * (r >> (1 - e))               # truncation toward zero
    if tie_fix:
        x = P - L * q
        q = np.where(x == 0, q & ~np.int64(1), q)
    assert np.abs(q).max(initial=0) < (1 << 15)  # the int16 halves of the pack
    return np.clip(q, 0, 255)


def _exact(P, L):
    n = P - L // 2
    q0 = np.floor_divide(n, L)
    r2 = 2 * (n - q0 * L)
    q = q0 + (r2 > L) + ((r2 == L) & (q0 % 2 == 1))
    return np.clip(q, 0, 255)


@pytest.mark.parametrize("name", NAMES)
def test_rounding_exhaustive_near_range(name):
    L, s, d = _params(name)
    assert d < 16000 and L % 2 == 0
    lo, hi = -2 * L, 258 * L
    step = 1 << 23
    for a in range(lo, hi, step):
        P = np.arange(a, min(a + step, hi), dtype=np.int64)
        got = _kernel_q(P, L, s, d)
        ref = _exact(P, L)
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, (name, int(P[bad[0]]), int(got[bad[0]]), int(ref[bad[0]]))


@pytest.mark.parametrize("name", NAMES)
def test_rounding_whole_range_sampled(name):
    L, s, d = _params(name)
    rng = np.random.default_rng(7)
    P = rng.integers(-2040 * L, 2040 * L + L // 2 + 1, size=1 << 20, dtype=np.int64)
    P = np.concatenate([P, np.array([-2040 * L + L // 2, 2040 * L + L // 2], dtype=np.int64)])
    assert np.array_equal(_kernel_q(P, L, s, d), _exact(P, L))


def test_ties_are_present_and_need_the_fix():
    """Every tie P = L q in range is hit, and without the remainder test the
    odd ones round the wrong way."""
    L, s, d = _params("T1")
    P = L * np.arange(0, 257, dtype=np.int64)
    assert np.array_equal(_kernel_q(P, L, s, d), _exact(P, L))
    wrong = _kernel_q(P, L, s, d, tie_fix=False) != _exact(P, L)
    assert wrong.sum() == 128                     # q = 1, 3, ..., 255


def test_offset_is_needed():
    """Planted mistake: without the 1/(2d) offset the truncation falls below
    exact multiples, so the check above has teeth."""
    L, s, d = _params("T1")
    P = np.arange(0, 40 * L, dtype=np.int64)
    inv = float(np.float32(1.0) / np.float32(d))
    q = np.trunc((P >> s).astype(np.float64) * inv).astype(np.int64)
    assert (np.clip(q, 0, 255) != np.floor_divide(P, L).clip(0, 255)).any()
