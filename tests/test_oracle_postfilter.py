"""Pins for the post-filter oracle (the filter is not in the paper, so these
are mathematical pins): bfloat16 rounding against torch, the convolution
against scipy's 2-D correlation and a brute-force loop, the adjoint identities
that define the two backward convolutions, finite differences of the float64
network, the identity filter, Adam's first step and the keep rule."""

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import postfilter as F
from synth import ar1_image, filter_params


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_param_count():
    assert F.N_PARAMS == 9857 == filter_params(0).size
    p = filter_params(3, bias_scale=0.1)
    assert np.array_equal(F.flatten(F.unflatten(p)), p.astype(np.float64))


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = _rng(1)
    x = rng.standard_normal(20000).astype(np.float32) * np.exp2(rng.integers(-20, 20, 20000))
    # exact ties: a bfloat16 value plus half of its unit in the last place
    base = F.bf16(rng.standard_normal(2000))
    _, e = np.frexp(base)
    ties = (base + np.sign(base) * np.ldexp(1.0, e - 9)).astype(np.float32)
    assert np.array_equal(ties.astype(np.float64), base + np.sign(base) * np.ldexp(1.0, e - 9))
    for v in (x, ties, np.array([0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 255.0, -128.0], np.float32)):
        ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(F.bf16(v.astype(np.float64)), ref)
    assert F.bf16(1 + 2 ** -8) == 1.0 and F.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def test_conv_matches_scipy_correlate():
    rng = _rng(2)
    a = rng.standard_normal((2, 3, 9, 11))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = F.conv3x3(a, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(a[n, i], w[o, i], mode="same", boundary="fill")
                             for i in range(3))
            np.testing.assert_allclose(out[n, o], ref, rtol=0, atol=1e-12)


def test_conv_bruteforce_loops():
    rng = _rng(3)
    a = rng.standard_normal((1, 2, 5, 4))
    w = rng.standard_normal((3, 2, 3, 3))
    out = F.conv3x3(a, w)
    for o in range(3):
        for y in range(5):
            for x in range(4):
                s = 0.0
                for i in range(2):
                    for dy in range(3):
                        for dx in range(3):
                            yy, xx = y + dy - 1, x + dx - 1
                            if 0 <= yy < 5 and 0 <= xx < 4:
                                s += w[o, i, dy, dx] * a[0, i, yy, xx]
                assert abs(out[0, o, y, x] - s) < 1e-12


def test_adjoint_identities():
    """<conv(a; w), g> = <a, input_grad(g; w)> = <w, weight_grad(g; a)>."""
    rng = _rng(4)
    a = rng.standard_normal((2, 5, 7, 6))
    w = rng.standard_normal((3, 5, 3, 3))
    g = rng.standard_normal((2, 3, 7, 6))
    lhs = np.sum(F.conv3x3(a, w) * g)
    assert abs(lhs - np.sum(a * F.conv3x3_input_grad(g, w))) < 1e-9 * abs(lhs) + 1e-9
    assert abs(lhs - np.sum(w * F.conv3x3_weight_grad(g, a))) < 1e-9 * abs(lhs) + 1e-9


def _pair(seed, h=16, w=16):
    orig = np.stack([ar1_image(h, w, 0.9, seed=seed + k) for k in range(2)])
    rng = _rng(seed)
    recon = np.clip(orig.astype(np.int64) + rng.integers(-6, 7, orig.shape), 0, 255).astype(np.uint8)
    return recon, orig


def test_gradient_central_differences():
    recon, orig = _pair(5)
    p = filter_params(7, last_scale=1.0, bias_scale=0.1).astype(np.float64)
    loss, g, _ = F.loss_and_grad(p, recon, orig, rounding=False)
    assert abs(loss - F.loss_only(p, recon, orig)) < 1e-15
    rng = _rng(6)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in F.LAYOUT])
    h = 1e-6
    for k in range(len(F.LAYOUT)):
        idx = rng.choice(np.arange(offsets[k], offsets[k + 1]), size=min(12, offsets[k + 1] - offsets[k]),
                         replace=False)
        for j in idx:
            pp, pm = p.copy(), p.copy()
            pp[j] += h
            pm[j] -= h
            fd = (F.loss_only(pp, recon, orig) - F.loss_only(pm, recon, orig)) / (2 * h)
            assert abs(fd - g[j]) <= 1e-6 * np.max(np.abs(g)) + 1e-6 * abs(g[j]), (F.LAYOUT[k][0], j)


def test_rounded_gradient_close_to_exact():
    recon, orig = _pair(8)
    p = filter_params(9, last_scale=1.0, bias_scale=0.05)
    _, g0, _ = F.loss_and_grad(p, recon, orig, rounding=False)
    _, g1, fw = F.loss_and_grad(p, recon, orig, rounding=True)
    assert np.linalg.norm(g1 - g0) < 0.05 * np.linalg.norm(g0)
    for k in ("w1", "w2", "w3", "a1", "a2"):
        assert np.array_equal(F.bf16(fw[k]), fw[k])


def test_zero_last_layer_is_identity():
    recon, orig = _pair(10)
    p = F.unflatten(filter_params(11, bias_scale=0.1))
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    res = F.apply(F.flatten(p), recon)
    assert np.array_equal(res["out"], recon)
    assert np.array_equal(res["y"], F.normalise(recon))


def test_adam_first_step_closed_form():
    rng = _rng(12)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = F.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=4e-15)   # 1 - 0.999 is not 0.001 exactly


def test_keep_rule():
    keep = F.keep_filtered([[10, 5, 5], [30, 0, 0], [0, 0, 0]], [[9, 6, 6], [29, 0, 0], [0, 0, 0]])
    assert keep.tolist() == [True, False, True]
