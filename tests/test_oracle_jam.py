"""Pins of the 16- and 32-point JAM matrices and the N-point transform coder (Sec. 6.2).

Anchors outside the oracle: the matrices and the cost table the paper prints,
the DCT-II closed form (the recursion applied to the exact 8-point DCT yields the
even rows of the exact 16-point DCT), and closed forms of the coder on inputs
whose reconstruction is known without a 2-D transform.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import codec, jam
from oracle import matrices as M
from synth import ar1_image

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _printed(n):
    rows = [l.split() for l in open(os.path.join(GOLD, f"jam_T{n}.txt")) if not l.startswith("#")]
    return np.array(rows, dtype=np.int64)


def _dct(n):
    """Orthonormal n-point DCT-II from its closed form."""
    k = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    c = np.cos((2 * x + 1) * k * math.pi / (2 * n)) * math.sqrt(2.0 / n)
    c[0] /= math.sqrt(2.0)
    return c


@pytest.mark.parametrize("n", [16, 32])
def test_matrices_are_the_printed_ones(n):
    assert np.array_equal(jam.jam_n(M.T1, n), _printed(n))


@pytest.mark.parametrize("n", [16, 32])
def test_recursion_as_written_differs_only_in_row_signs(n):
    t = jam.jam_n(M.T1, n // 2)
    lit = jam.jam_as_written(t)
    ours = jam.jam(t)
    flipped = [k for k in range(n) if not np.array_equal(lit[k], ours[k])]
    for k in flipped:
        assert np.array_equal(lit[k], -ours[k])
    # exactly the odd rows grown from an antisymmetric row of the half-size matrix
    expect = [2 * i + 1 for i in range(n // 2) if np.array_equal(t[i], -t[i, ::-1])]
    assert flipped == expect and len(expect) > 0


@pytest.mark.parametrize("n", [16, 32])
def test_row_norms_are_the_kronecker_forms(n):
    t = jam.jam_n(M.T1, n)
    g = t @ t.T
    assert np.count_nonzero(g - np.diag(np.diag(g))) == 0          # orthogonal rows
    assert np.array_equal(np.diag(g), jam.d_kron(n))
    gold = json.load(open(os.path.join(GOLD, "jam_cost.json")))
    assert "kron" in gold["D_16"] and "kron" in gold["D_32"]


def test_cost_table():
    gold = json.load(open(os.path.join(GOLD, "jam_cost.json")))["proposed"]
    for n in (8, 16, 32):
        assert jam.jam_cost(n) == (gold[str(n)]["adds"], gold[str(n)]["shifts"])


@pytest.mark.parametrize("n", [16, 32])
def test_fast_recursion_is_the_matrix(n):
    rng = np.random.default_rng(n)
    x = rng.integers(-(1 << 20), 1 << 20, size=(20_000, n))
    y = np.stack(jam.jam_fast([x[:, k] for k in range(n)], n), axis=1)
    assert np.array_equal(y, x @ jam.jam_n(M.T1, n).T)


@pytest.mark.parametrize("builder", [jam.jam, jam.jam_as_written])
def test_recursion_on_the_exact_dct_gives_its_even_rows(builder):
    # C_(2h) rows 2i are (1/sqrt 2)[c_i, rev(c_i)] for the DCT-II: the recursion,
    # with its 1/sqrt 2, applied to the exact h-point DCT reproduces them
    for h in (8, 16):
        big = builder(_dct(h)) / math.sqrt(2.0)
        assert np.allclose(big[0::2], _dct(2 * h)[0::2], atol=1e-14)


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("shape", [(64, 96), (70, 45), (5, 3)])
def test_full_retention_is_lossless(n, shape):
    img = ar1_image(*shape, rho=0.9, seed=sum(shape))
    out = jam.evaluate(img, jam.jam_n(M.T1, n), n * n, 0)
    assert out["sse"] == 0 and np.array_equal(out["rec"], img)


def _extend(img, n):
    """Repeat the last row and column up to multiples of n, by clamped indexing."""
    h, w = img.shape
    ys = np.minimum(np.arange(-(-h // n) * n), h - 1)
    xs = np.minimum(np.arange(-(-w // n) * n), w - 1)
    return np.asarray(img, dtype=np.int64)[ys][:, xs]


def _block_means_rne(img, n, num_fn):
    big = _extend(img, n)
    h, w = big.shape
    s = big.reshape(h // n, n, w // n, n).sum(axis=(1, 3))
    q = num_fn(s)
    return np.repeat(np.repeat(q, n, 0), n, 1)[: img.shape[0], : img.shape[1]]


@pytest.mark.parametrize("n", [16, 32])
def test_dc_only_is_the_block_mean(n):
    # row 0 of T_(n) is all ones: with r = 1 each pixel is the rounded mean of
    # its (edge-extended) block
    img = ar1_image(77, 101, rho=0.95, seed=4)
    out = jam.evaluate(img, jam.jam_n(M.T1, n), 1, 0)
    want = _block_means_rne(img, n, lambda s: codec.rne_div(s, n * n))
    assert np.array_equal(out["rec"], want)


@pytest.mark.parametrize("n,step", [(16, 16), (16, 48), (32, 32), (32, 96)])
def test_dc_only_quantised(n, step):
    # B(0, 0) = block sum / n; q = round-half-away(B / step); each pixel is
    # step q / n rounded half to even
    img = ar1_image(96, 64, rho=0.95, seed=9)
    out = jam.evaluate(img, jam.jam_n(M.T1, n), 1, step)

    def f(s):
        q = (2 * s + n * step) // (2 * n * step)              # s >= 0
        return np.clip(codec.rne_div(step * q, n), 0, 255)
    assert np.array_equal(out["rec"], _block_means_rne(img, n, f))
    assert np.array_equal(out["coef_int"][:, 0],
                          ((2 * _extend(img, n).reshape(96 // n, n, 64 // n, n)
                            .sum(axis=(1, 3)) + n * step) // (2 * n * step)).ravel())


@pytest.mark.parametrize("n", [16, 32])
def test_orientation_with_two_coefficients(n):
    # the second zig-zag coefficient is (0, 1): horizontal frequency 1.  An image
    # that varies only across columns keeps its 1-D projection on rows 0 and 1 of
    # C_hat; one that varies only down the rows keeps just its block means.
    from fractions import Fraction
    t = jam.jam_n(M.T1, n)
    nrm = np.sum(t * t, axis=1)
    rng = np.random.default_rng(1)
    prof = rng.integers(0, 256, size=2 * n)
    cols = np.tile(prof, (n, 1)).astype(np.uint8)              # n x 2n, varies along x
    out = jam.evaluate(cols, t, 2, 0)
    want = []
    for b in range(2):
        p = prof[b * n:(b + 1) * n]
        for x in range(n):   # exact: sum over k < 2 of t_k[x] (t_k . p) / n_k
            v = sum(Fraction(int(t[k, x]) * int(t[k] @ p), int(nrm[k])) for k in range(2))
            want.append(min(max(round(v), 0), 255))           # Fraction rounds half to even
    assert out["rec"][0].tolist() == want
    rows = np.ascontiguousarray(cols.T)                         # 2n x n, varies along y
    out = jam.evaluate(rows, t, 2, 0)
    want = _block_means_rne(rows, n, lambda s: codec.rne_div(s, n * n))
    assert np.array_equal(out["rec"], want)


@pytest.mark.parametrize("n,step", [(16, 16), (32, 32)])
def test_quantised_levels_against_the_real_transform(n, step):
    # the exact-arithmetic levels equal round-half-away of the float64
    # B = C_hat A C_hat^T over step, away from float ties
    t = jam.jam_n(M.T1, n)
    c = t / np.sqrt(np.sum(t * t, axis=1))[:, None]
    img = ar1_image(4 * n, 3 * n, rho=0.93, seed=n)
    r = n * n // 4
    out = jam.evaluate(img, t, r, step)
    blocks = codec.to_blocks(img, n).astype(np.float64)
    b = np.einsum("ki,bij,lj->bkl", c, blocks, c) / step
    zz = codec.zigzag(n)[:r]
    v = np.stack([b[:, k, l] for k, l in zz], axis=1)
    frac = np.abs(np.abs(v) - np.floor(np.abs(v)) - 0.5)
    far = frac > 1e-9
    want = np.sign(v) * np.floor(np.abs(v) + 0.5)
    assert far.mean() > 0.99
    assert np.array_equal(out["coef_int"][far], want[far].astype(np.int64))
    near = ~far
    assert np.array_equal(out["coef_int"][near], (np.sign(v) * np.ceil(np.abs(v) - 1e-9))[near].astype(np.int64))


@pytest.mark.parametrize("n", [16, 32])
def test_constant_image_any_size(n):
    for shape in ((1, 1), (17, 33), (40, 24)):
        img = np.full(shape, 77, dtype=np.uint8)
        for r in (1, 3, n * n):
            assert np.array_equal(jam.evaluate(img, jam.jam_n(M.T1, n), r, 0)["rec"], img)


def _two_level_blocks(n, seed):
    """Blocks whose left half is a and right half b (a + b and a - b odd)."""
    rng = np.random.default_rng(seed)
    nb = 6
    a = rng.integers(0, 128, size=nb) * 2 + 1          # odd
    b = rng.integers(0, 128, size=nb) * 2              # even
    img = np.zeros((n, nb * n), dtype=np.uint8)
    for i in range(nb):
        img[:, i * n:i * n + n // 2] = a[i]
        img[:, i * n + n // 2:(i + 1) * n] = b[i]
    return img, a.astype(np.int64), b.astype(np.int64)


@pytest.mark.parametrize("n", [16, 32])
def test_quantiser_ties_round_away_from_zero(n):
    # B(0, 0) = n (a + b) / 2 and B(0, 1) = n (a - b) / 2 (rows 0 and 1 of T_(n)
    # are all ones and n/2 ones then n/2 minus ones, both of norm n): with step n
    # both quotients are exact halves, of either sign
    img, a, b = _two_level_blocks(n, seed=n)
    out = jam.evaluate(img, jam.jam_n(M.T1, n), 2, n)
    away = lambda num: np.sign(num) * ((np.abs(num) + 1) // 2)     # num odd: num / 2 away from 0
    assert np.array_equal(out["coef_int"][:, 0], away(a + b))
    assert np.array_equal(out["coef_int"][:, 1], away(a - b))
