"""Independent pins of the oracle's QUANTISED 8x8 decode (Sec. 6.1.1 inverse
C_hat^T B' C_hat applied to the dequantised coefficients B' = step q).

Three checks, none of which reuses the oracle's inverse arithmetic:

* Parseval with quantisation: C_hat is orthonormal, so the unrounded
  reconstruction error of a block equals its coefficient-domain error, the kept
  coefficients' (B - step q)^2 plus the dropped coefficients' B^2.  A transposed
  C_hat, a wrong dequantisation scale or a wrong orientation of the inverse all
  break this identity.
* An exact restatement: every reconstructed pixel is a finite sum
  sum_kl T[k,x] T[l,y] step q_kl / sqrt(n_k n_l), an element of a multiquadratic
  field Q(sqrt 2, sqrt 3, sqrt 5, ...).  Writing n_k n_l = c^2 s with s
  square-free, each term is a rational multiple of sqrt(s), and the sign of any
  element of such a field is decidable exactly (split off the largest prime p,
  x + sqrt(p) y, and compare x^2 with p y^2 one field down).  Round-half-to-even
  and clipping are then exact integer decisions, compared pixel for pixel with
  the oracle's decode.
* Ties: levels built so that the exact value is a half (it must go to the even
  neighbour) or lies within ~1e-8 of a half, where float64 alone cannot decide.
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import codec as Co
from oracle import matrices as M
from synth import ar1_image

INT_T = ["T1", "T2", "LO", "T6", "RDCT", "T4"]


# ----------------------------------------------------------------- exact field arithmetic

def _squarefree(n: int) -> tuple[int, tuple[int, ...]]:
    """n = c^2 * prod(primes) with distinct primes: returns (c, primes)."""
    c, primes, p = 1, [], 2
    while p * p <= n:
        e = 0
        while n % p == 0:
            n //= p
            e += 1
        c *= p ** (e // 2)
        if e % 2:
            primes.append(p)
        p += 1
    if n > 1:
        primes.append(n)
    return c, tuple(sorted(primes))


def _mul(a: dict, b: dict) -> dict:
    """Product of two field elements {primes: coefficient} (value sum c sqrt(prod primes))."""
    out: dict = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            sa, sb = set(ka), set(kb)
            f = math.prod(sa & sb)
            key = tuple(sorted(sa ^ sb))
            out[key] = out.get(key, 0) + va * vb * f
    return {k: v for k, v in out.items() if v != 0}


def _sign(a: dict) -> int:
    a = {k: v for k, v in a.items() if v != 0}
    if not a:
        return 0
    primes = sorted({p for k in a for p in k})
    if not primes:
        v = a[()]
        return (v > 0) - (v < 0)
    p = primes[-1]
    x = {k: v for k, v in a.items() if p not in k}
    y = {tuple(q for q in k if q != p): v for k, v in a.items() if p in k}   # a = x + sqrt(p) y
    sx, sy = _sign(x), _sign(y)
    if sy == 0:
        return sx
    if sx == 0 or sx == sy:
        return sy if sx == 0 else sx
    d = _mul(x, x)
    for k, v in _mul(y, y).items():
        d[k] = d.get(k, 0) - p * v
    return sx * _sign(d)                      # |x| > sqrt(p)|y| iff x^2 - p y^2 > 0


def _exact_pixels(t: np.ndarray, q_zz: np.ndarray, r: int, step: int) -> np.ndarray:
    """Exact rne + clip of sum_kl T[k,x] T[l,y] step q_kl / sqrt(n_k n_l) for one block."""
    t = np.asarray(t, dtype=np.int64)
    n = [int(v) for v in (t * t).sum(axis=1)]
    zz = Co.zigzag()[:r]
    out = np.zeros((8, 8), dtype=np.int64)
    terms = []
    for p, (k, l) in enumerate(zz):
        qv = int(q_zz[p])
        if qv == 0:
            continue
        c, s = _squarefree(n[k] * n[l])
        # 1 / (c sqrt(S)) = sqrt(S) / (c S)
        terms.append((k, l, Fraction(step * qv, c * math.prod(s)), s))
    for x in range(8):
        for y in range(8):
            a: dict = {}
            for k, l, f, s in terms:
                w = int(t[k, x] * t[l, y])
                if w:
                    a[s] = a.get(s, 0) + w * f
            approx = sum(float(v) * math.sqrt(math.prod(k)) for k, v in a.items())
            m = math.floor(approx)

            def cmp(c: Fraction) -> int:
                b = dict(a)
                b[()] = b.get((), 0) - c
                return _sign(b)

            while cmp(Fraction(m)) < 0:
                m -= 1
            while cmp(Fraction(m + 1)) >= 0:
                m += 1
            h = cmp(Fraction(2 * m + 1, 2))
            v = m + 1 if h > 0 or (h == 0 and m % 2 == 1) else m
            out[x, y] = min(max(v, 0), 255)
    return out


def test_field_sign_helpers():
    # sqrt(10) - 3 > 0; 19 - 6 sqrt(10) > 0 (361 > 360); 4443 - 1405 sqrt(10) < 0
    # (4443^2 = 19,740,249 < 10 * 1405^2 = 19,740,250)
    assert _sign({(2, 5): 1, (): -3}) == 1
    assert _sign({(): 19, (2, 5): -6}) == 1
    assert _sign({(): 4443, (2, 5): -1405}) == -1
    assert _sign({(): -4443, (2, 5): 1405}) == 1
    # sqrt(2) + sqrt(3) - sqrt(10) = -0.0166; sqrt(6) - sqrt(2) - sqrt(3) = -0.697
    assert _sign({(2,): 1, (3,): 1, (2, 5): -1}) == -1
    assert _sign({(2, 3): 1, (2,): -1, (3,): -1}) == -1
    # (sqrt 2 + sqrt 3)^2 = 5 + 2 sqrt 6: exactly zero against its expansion
    sq = _mul({(2,): 1, (3,): 1}, {(2,): 1, (3,): 1})
    assert sq == {(): 5, (2, 3): 2}
    assert _sign({**sq, (): 0, (2, 3): 0}) == 0
    assert _mul({(2,): 1}, {(2,): 1}) == {(): 2}
    assert _squarefree(160) == (4, (2, 5)) and _squarefree(400) == (20, ())


# ----------------------------------------------------------------- Parseval with quantisation

@pytest.fixture(scope="module")
def img():
    return ar1_image(48, 64, 0.95, seed=21)


@pytest.mark.parametrize("name", INT_T)
@pytest.mark.parametrize("r", [6, 10, 21, 64])
@pytest.mark.parametrize("step", [8, 16, 40])
def test_parseval_quantised(img, name, r, step):
    t = M.TRANSFORMS[name]
    res = Co.evaluate(img, t, r, step)
    blocks = Co.to_blocks(img)
    b_all = Co.take_zigzag(Co.scale_coeffs(Co.forward_int(blocks, t), t), 64)
    q = np.asarray(res["coef_int"], dtype=np.float64)
    coeff_err = float(np.sum((b_all[:, :r] - step * q) ** 2) + np.sum(b_all[:, r:] ** 2))
    pix_err = float(np.sum((img.astype(np.float64) - res["real"]) ** 2))
    assert abs(pix_err - coeff_err) <= 1e-9 * max(coeff_err, 1.0), (pix_err, coeff_err)


def test_parseval_catches_a_transposed_inverse(img):
    """The identity above is not vacuous: decoding with C_hat A C_hat^T (the
    forward orientation) instead of C_hat^T B C_hat changes the error energy."""
    t, r, step = M.T1, 10, 16
    enc = Co.encode(img, t, r, step)
    c_hat = M.approx_matrix(t)
    bq = Co.put_zigzag(enc["coef_int"].astype(np.float64) * step, r, np.float64)
    wrong = Co.from_blocks(np.einsum("ik,bkl,jl->bij", c_hat, bq, c_hat), *img.shape)
    right = Co.decode(enc["coef_int"], t, r, *img.shape, step)["real"]
    e_wrong = float(np.sum((img - wrong) ** 2))
    e_right = float(np.sum((img - right) ** 2))
    assert abs(e_wrong - e_right) > 1e-3 * e_right


# ----------------------------------------------------------------- exact restatement

@pytest.mark.parametrize("name", INT_T)
@pytest.mark.parametrize("step", [8, 16, 40])
def test_quantised_decode_equals_exact_field_rounding(name, step):
    """AR(1) blocks at the quantiser steps the library accepts: every pixel of
    the oracle's decode equals the exactly rounded reconstruction."""
    t = M.TRANSFORMS[name]
    img = ar1_image(32, 64, 0.9, seed=5)
    r = 21
    res = Co.evaluate(img, t, r, step)
    rec_blocks = Co.to_blocks(res["rec"])
    for b in range(rec_blocks.shape[0]):
        assert np.array_equal(rec_blocks[b], _exact_pixels(t, res["coef_int"][b], r, step)), (name, b)


@pytest.mark.parametrize("name", ["T1", "T2", "T6", "RDCT", "T4", "LO"])
@pytest.mark.parametrize("step", [5, 12])
def test_quantised_decode_exact_at_general_steps(name, step):
    """Random levels at steps where the rational part of a reconstruction can
    be an exact half (5 and 12 are not multiples of 8): half the blocks carry
    levels only on coefficients whose n_k n_l is a perfect square, so their
    pixels are rational and hit exact halves often."""
    t = M.TRANSFORMS[name]
    n = M.row_norms2(t)
    zi, zj = Co.zz_index_arrays()
    r = 36
    rational = np.array([math.isqrt(int(n[zi[p]] * n[zj[p]])) ** 2 == int(n[zi[p]] * n[zj[p]])
                         for p in range(r)])
    rng = np.random.Generator(np.random.PCG64(7))
    nb = 96
    q = rng.integers(-6, 7, size=(nb, r))
    q[:, 0] = rng.integers(0, 40, size=nb)
    q[: nb // 2, ~rational] = 0
    dec = Co.decode(q, t, r, 8, 8 * nb, step)
    got = Co.to_blocks(dec["rec"])
    for b in range(nb):
        assert np.array_equal(got[b], _exact_pixels(t, q[b], r, step)), (name, step, b)
    real = dec["real"]
    halves = int(np.sum(np.abs(real - np.floor(real) - 0.5) < 1e-9))
    assert halves > 0           # the case this test is for actually occurs


def test_exact_half_rounds_to_even():
    """T1, step 5, DC level 4 only: every pixel is exactly 5 * 4 / 8 = 2.5 and
    rounds to 2; DC level 12 gives 7.5, which rounds to 8."""
    for level, want in ((4, 2), (12, 8), (-4, 0)):
        q = np.zeros((1, 1), dtype=np.int64)
        q[0, 0] = level
        rec = Co.decode(q, M.T1, 1, 8, 8, 5)["rec"]
        assert np.all(rec == want), (level, rec)


def _sqrt10_convergents(count: int):
    """Convergents p/b of sqrt(10) = [3; 6, 6, 6, ...]."""
    p0, b0, p1, b1 = 1, 0, 3, 1
    out = []
    for _ in range(count):
        p0, b0, p1, b1 = p1, b1, 6 * p1 + p0, 6 * b1 + b0
        out.append((p1, b1))
    return out


def test_near_half_decided_exactly():
    """T1 at step 20 with levels q_00 and q_02 only: at a pixel where
    T[0,x] T[2,y] = 1 the value is 20 q_00 / 8 + 20 q_02 / sqrt(160)
    = 2.5 q_00 + q_02 sqrt(10) / 2.  With q_02 = b, p/b a convergent of
    sqrt(10) with p odd, q_02 sqrt(10) / 2 lies within |b sqrt(10) - p| / 2 of
    the half p / 2, and q_00 moves the result to a target in [248.5, 252.5]:
    the pixel lies 1e-9 to 1e-5 from that half, and for the largest levels
    below the spacing of float64 at the magnitude of the terms (~1e8).  The
    decode must agree with the exact decision at every pixel."""
    cases = 0
    for p, b in _sqrt10_convergents(11):
        if p % 2 == 0 or b < 10 ** 4:
            continue
        for target2 in (497, 499, 501, 503, 505):      # 2 x target, one per residue mod 5
            num = target2 - p                          # 5 q00 = 2 target - p
            if num % 10:
                continue
            q00 = num // 5
            r = 6                                      # (0, 2) is zig-zag position 5
            q = np.zeros((1, r), dtype=np.int64)
            q[0, 0] = q00
            q[0, 5] = b
            dec = Co.decode(q, M.T1, r, 8, 8, 20)
            assert abs(dec["real"][0, 1] - target2 / 2) < 1e-4, dec["real"][0, 1]
            want = _exact_pixels(M.T1, q[0], r, 20)
            assert np.array_equal(dec["rec"], want), (p, b, target2)
            cases += 1
    assert cases >= 4
