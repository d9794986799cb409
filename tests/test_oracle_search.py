"""Pins of the greedy angle-similarity search (Sec. 3, Sec. 4.1)."""

import json
import math
import os

import numpy as np
import pytest

from oracle import ctuples
from oracle import matrices as M
from oracle import measures as Me
from oracle import search as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NAMES = {"RDCT": M.T_RDCT, "T4": M.T4, "T1": M.T1, "T2": M.T2}


def _names(mats):
    out = []
    for m in mats:
        hit = [n for n, t in NAMES.items() if np.array_equal(t, m)]
        out.append(hit[0] if hit else "other")
    return sorted(out)


def test_search_space_sizes():
    # |D1| = 6,561 and |D2| = 390,625 (Sec. 3.2); zero vector excluded here
    assert len(S.search_space(S.P1)[0]) == 3 ** 8 - 1
    assert len(S.search_space(S.P2)[0]) == 5 ** 8 - 1
    d, idx = S.search_space(S.P1, include_zero=True)
    assert np.array_equal(d[0], np.zeros(8)) and np.array_equal(idx, np.arange(3 ** 8))


def test_closure_d1_720_orders():
    gold = json.load(open(os.path.join(GOLD, "search_results.json")))
    mats, leaves, dead = S.closure(S.P1)
    assert _names(mats) == sorted(gold["D1_720_orders"])
    assert dead == 0


def test_worked_examples_d1():
    gold = json.load(open(os.path.join(GOLD, "search_results.json")))
    fwd, _, _ = S.closure(S.P1, orders=[tuple(range(8))], fixed=None)
    rev, _, _ = S.closure(S.P1, orders=[tuple(range(7, -1, -1))], fixed=None)
    assert gold["worked_order_forward"] in _names(fwd)
    assert gold["worked_order_reverse"] in _names(rev)


@pytest.mark.slow
def test_closure_d2_720_orders():
    gold = json.load(open(os.path.join(GOLD, "search_results.json")))
    mats, leaves, dead = S.closure(S.P2)
    assert _names(mats) == sorted(gold["D2_720_orders"])
    assert leaves == 240


def test_canonical_orders_land_in_closure():
    rng = np.random.default_rng(1)
    perms = [tuple(rng.permutation(list(S.FREE_ROWS))) for _ in range(12)]
    space = S._Space(S.P1)
    for o in perms:
        t = S.greedy_canonical(S.P1, o, space=space)
        assert t is not None and _names([t])[0] in ("RDCT", "T4")
        assert M.is_orthogonal_rows(t)


def test_t1_live_orders_d2():
    # two orders reported live for T1 by the closure (canonical form agrees)
    space = S._Space(S.P2)
    for o in [(1, 2, 6, 7, 3, 5), (1, 2, 7, 3, 5, 6)]:
        t = S.greedy_canonical(S.P2, o, space=space)
        assert t is not None and np.array_equal(t, M.T1)


def test_identity_order_d2_is_dead():
    assert S.greedy_canonical(S.P2, (1, 2, 3, 5, 6, 7)) is None


def test_t1_row_angles_and_error_energy():
    ang = S.row_angles_deg(M.T1)
    expect = [0, 9.8516, 4.0651, 23.0411, 0, 23.0411, 4.0651, 9.8516]
    np.testing.assert_allclose(ang, expect, atol=1e-4)
    eps = math.pi * np.sum(2 * (1 - np.cos(np.radians(ang))))
    assert round(eps, 4) == 1.2194          # Sec. 4.3 measures table


def test_tuples_c_matches_python():
    rng = np.random.default_rng(5)
    lists = [rng.integers(-1, 2, size=(6, 8)) for _ in range(8)]
    lists[0][0] = 1
    py = S.orthogonal_tuples_py(lists)
    c, n = ctuples.orthogonal_tuples(lists)
    assert n == len(py)
    assert [tuple(r) for r in c] == py


def test_tuples_recover_t1_from_its_rows():
    # each list holds T1's row plus decoys; the only orthogonal tuple is T1
    rng = np.random.default_rng(9)
    lists = []
    for k in range(8):
        decoy = rng.integers(-2, 3, size=(5, 8))
        lists.append(np.vstack([decoy[:2], M.T1[k], decoy[2:]]))
    tups, n = ctuples.orthogonal_tuples(lists)
    rows = [np.stack([lists[k][tp[k]] for k in range(8)]) for tp in tups]
    assert any(np.array_equal(r, M.T1) for r in rows)
    assert all(M.is_orthogonal_rows(r) for r in rows)


def test_topk_small_space_brute_force():
    # top-k of P2 by the chunked scan equals a direct sort of the whole space
    res = S.topk_scan(S.P2, 20, chunk=50_000)
    d, idx = S.search_space(S.P2)
    prim = S._gcd_rows(d) == 1
    d, idx = d[prim], idx[prim]
    c = M.dct_matrix()
    for row in range(8):
        cos = S.cosines(d, c[row])
        order = S.canonical_order(cos, np.sum(d * d, axis=1), idx)[:20]
        assert np.array_equal(res[row]["idx"], idx[order])
    assert np.array_equal(res[2]["vec"][0], M.T1[2])


def _brute_greedy_ok(p, order, t):
    """Check a full-order greedy result by plain loops: every row is orthogonal
    to the rows chosen before it, and no vector of P^8 orthogonal to them has a
    strictly larger cosine to its DCT row (beyond the tie tolerance)."""
    import itertools
    c = M.dct_matrix()
    chosen = []
    for k in order:
        best = -2.0
        for v in itertools.product(p, repeat=8):
            if not any(v):
                continue
            if any(sum(a * b for a, b in zip(v, u)) for u in chosen):
                continue
            cs = sum(a * b for a, b in zip(v, c[k])) / math.sqrt(sum(a * a for a in v))
            best = max(best, cs)
        row = [int(x) for x in t[k]]
        if any(sum(a * b for a, b in zip(row, u)) for u in chosen):
            return False
        got = sum(a * b for a, b in zip(row, c[k])) / math.sqrt(sum(a * a for a in row))
        if got < best - S.TIE_EPS:
            return False
        chosen.append(row)
    return True


def test_full_order_greedy_by_brute_force():
    """All eight rows free (the 8! orders of Sec. 3.5): a few orders on D1
    checked against exhaustive loops."""
    rng = np.random.default_rng(5)
    space = S._Space(S.P1)
    for _ in range(3):
        o = [int(x) for x in rng.permutation(8)]
        t = S.greedy_canonical(S.P1, o, fixed=None, space=space)
        assert t is not None and _brute_greedy_ok(S.P1, o, t)


def test_full_order_closure_d1_is_rdct_and_t4():
    """Without fixed rows the closure over all 40,320 orders on D1 reaches the
    same two matrices as the 720-order search of Sec. 4.1."""
    mats, leaves, dead = S.closure(S.P1, orders=None, fixed=None)
    keys = sorted(np.asarray(m, dtype=np.int8).tobytes() for m in mats)
    assert keys == sorted(np.asarray(m, dtype=np.int8).tobytes() for m in (M.T_RDCT, M.T4))
    assert leaves >= 40320 and dead == 0


@pytest.mark.parametrize("p", [(0, 1, -1, 4, -4), (0, 1, -1, 8, -8)])
def test_extended_sets_do_not_beat_t1(p):
    """Sec. 4.1: the extended entry sets gave matrices that performed worse than
    the proposed ones at a higher cost.  For the five-element sets: every matrix
    of the 720-order closure has a lower coding gain and transform efficiency
    than T1, and more additions and more non-trivial multiplications (entries
    other than 0 and +-1) in direct form."""
    mats, leaves, dead = S.closure(p)
    assert len(mats) >= 1 and leaves == 720
    ref = Me.measures(M.T1)

    def cost(t):
        t = np.asarray(t)
        return (int(sum(max(np.count_nonzero(r) - 1, 0) for r in t)),
                int(np.count_nonzero(np.abs(t) > 1)))
    for t in mats:
        m = Me.measures(t)
        assert m["cg_star"] < ref["cg_star"] and m["eta"] < ref["eta"]
        assert cost(t)[0] > cost(M.T1)[0] and cost(t)[1] > cost(M.T1)[1]
