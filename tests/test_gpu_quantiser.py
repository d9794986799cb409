"""Exhaustive GPU check of the quantiser (reading 6: q = round-half-away(B / step),
B = s_k s_l Y): for one coefficient of every scale class n_k n_l of each
transform, 8-bit blocks are built whose integer stage Y_kl takes EVERY value
the class can reach over 8-bit input, and the levels the library writes are
compared with the oracle's for all retained coefficients of those blocks.

A block reaching a given Y_kl = sum_x T[k,x] (sum_y T[l,y] A[x,y]) is found in
two greedy steps: the outer sum picks row values R_x in their reachable range,
then each row's pixels are picked so that sum_y T[l,y] A[x,y] = R_x.  Every row
of the matrices has a +-1 entry, so both steps can hit any integer in range;
the construction is checked by recomputing Y with the oracle."""

import math

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import codec as Co
from oracle import matrices as M


def _solve(weights, lo, hi, targets):
    """Integer v (n, len(weights)) with lo <= v <= hi and v @ weights == targets."""
    w = np.asarray(weights, dtype=np.int64)
    n = targets.shape[0]
    v = np.where(w > 0, lo, hi).astype(np.int64)
    v = np.where(w == 0, 0 if lo <= 0 <= hi else lo, v)
    v = np.broadcast_to(v, (n, w.size)).copy()
    d = targets - v @ w
    assert np.all(d >= 0)
    for i in np.argsort(-np.abs(w), kind="stable"):
        if w[i] == 0:
            continue
        take = np.minimum(d // abs(w[i]), hi - lo)
        v[:, i] += np.sign(w[i]) * take
        d -= take * abs(w[i])
    assert np.all(d == 0)
    return v


def _range(weights, lo, hi):
    w = np.asarray(weights, dtype=np.int64)
    return int(np.sum(np.where(w > 0, w * lo, w * hi))), int(np.sum(np.where(w > 0, w * hi, w * lo)))


def sweep_blocks(t, k, l):
    """(nb, 8, 8) uint8 blocks with Y_kl running over its whole reachable range
    (the multiples of g_k g_l, g the gcd of a row's entries, between the
    extremes)."""
    t = np.asarray(t, dtype=np.int64)
    gk, gl = math.gcd(*t[k]), math.gcd(*t[l])
    wk, wl = t[k] // gk, t[l] // gl
    rlo, rhi = _range(wl, 0, 255)
    ylo, yhi = _range(wk, rlo, rhi)
    targets = np.arange(ylo, yhi + 1, dtype=np.int64) * gk * gl
    rows = _solve(wk, rlo, rhi, targets // (gk * gl))            # R_x / g_l
    blocks = np.empty((targets.size, 8, 8), dtype=np.int64)
    for x in range(8):
        blocks[:, x, :] = _solve(wl, 0, 255, rows[:, x])
    y = Co.forward_int(blocks, t)
    assert np.array_equal(y[:, k, l], targets)
    return blocks.astype(np.uint8), targets


def class_representatives(t, r):
    n = M.row_norms2(t)
    seen, reps = set(), []
    for k, l in Co.zigzag()[:r]:
        c = int(n[k] * n[l])
        if c not in seen:
            seen.add(c)
            reps.append((k, l, c))
    return reps


CASES = [("T1", 8), ("T1", 16), ("T1", 40), ("T2", 16), ("T6", 16), ("RDCT", 16), ("T4", 16),
         ("LO", 32), ("LO", 64)]


def test_sweep_construction_cpu():
    """The block builder reaches every Y of T1's DC and of 360- and 400-class
    coefficients, and every multiple of 4 of the doubled LO's DC; every class of
    every transform sits in the first 13 zig-zag positions."""
    b, y = sweep_blocks(M.T1, 0, 0)
    assert y[0] == 0 and y[-1] == 64 * 255 and b.shape[0] == 16321
    b, y = sweep_blocks(M.T1, 1, 2)        # rows 1 and 2 have +-5 and +-6 entry sums
    assert y[0] == -y[-1] and y[-1] == 255 * (5 * 6 + 5 * 6) and b.shape[0] == 2 * 15300 + 1
    b, y = sweep_blocks(M.T1, 2, 2)        # the largest |Y| of T1 over 8-bit blocks
    assert y[0] == -18360 and y[-1] == 18360
    b, y = sweep_blocks(M.T_LO_X2, 0, 0)
    assert y[-1] == 4 * 64 * 255 and b.shape[0] == 16321
    for name, t in M.TRANSFORMS.items():
        n = M.row_norms2(t)
        assert {c for _, _, c in class_representatives(t, 13)} == {int(a * b) for a in n for b in n}


@pytest.mark.gpu
@pytest.mark.parametrize("name,step", CASES)
def test_quantiser_every_reachable_level(cuda, name, step):
    import torch
    t = M.TRANSFORMS[name]
    r = 13                                   # the first 13 zig-zag positions hold every class
    reps = class_representatives(t, r)
    for k, l, c in reps:
        blocks, _ = sweep_blocks(t, k, l)
        nb = blocks.shape[0]
        img = np.ascontiguousarray(blocks.transpose(1, 0, 2).reshape(8, 8 * nb))
        d = torch.from_numpy(img).to(cuda)
        got, _ = A.encode_blocks(d, name, r, step)
        y = Co.take_zigzag(Co.forward_int(blocks.astype(np.int64), t), r)
        want = Co.quantize(y, t, r, step)
        g = got.cpu().numpy().astype(np.int64)
        bad = np.argwhere(g != want)
        assert bad.size == 0, (name, step, (k, l, c), bad[:5], g[tuple(bad[0])], want[tuple(bad[0])])
