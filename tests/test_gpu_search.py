"""GPU angle search (through the C ABI) against the oracle's greedy search,
top-k scan and tuple enumeration: matrices, counts, argmin indices and
tuples bit-exact."""

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import ctuples
from oracle import matrices as M
from oracle import search as S

pytestmark = pytest.mark.gpu


def _key(m):
    return np.asarray(m, dtype=np.int8).tobytes()


def test_closure_d1_720(cuda):
    mats, ang, leaves, dead = A.derive_transform(S.P1, A.SEARCH_CLOSURE)
    ref, rleaves, rdead = S.closure(S.P1)
    assert [_key(m) for m in mats] == [_key(m) for m in ref]
    assert (leaves, dead) == (rleaves, rdead)
    assert sorted(_key(m) for m in mats) == sorted([_key(M.T_RDCT), _key(M.T4)])


def test_closure_d2_720(cuda):
    mats, ang, leaves, dead = A.derive_transform(S.P2, A.SEARCH_CLOSURE)
    ref, rleaves, rdead = S.closure(S.P2)
    assert [_key(m) for m in mats] == [_key(m) for m in ref]
    assert (leaves, dead) == (rleaves, rdead)
    assert sorted(_key(m) for m in mats) == sorted([_key(M.T1), _key(M.T2)])
    i1 = [_key(m) for m in mats].index(_key(M.T1))
    # arccos near 1 turns a one-ulp cosine difference into ~1e-6 degrees
    np.testing.assert_allclose(np.cos(ang[i1]), np.cos(np.radians(S.row_angles_deg(M.T1))),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.degrees(ang[i1]), S.row_angles_deg(M.T1), atol=2e-6)


def test_worked_orders_without_fixed_rows(cuda):
    for order in (list(range(8)), list(range(7, -1, -1))):
        mats, _, leaves, dead = A.derive_transform(S.P1, A.SEARCH_CLOSURE, orders=[order],
                                                   fix_rows_1_5=False)
        ref, rl, rd = S.closure(S.P1, orders=[tuple(order)], fixed=None)
        assert [_key(m) for m in mats] == [_key(m) for m in ref]
        assert (leaves, dead) == (rl, rd)


def test_canonical_per_order_d2(cuda):
    rng = np.random.default_rng(7)
    orders = [tuple(rng.permutation(list(S.FREE_ROWS))) for _ in range(24)]
    orders += [(1, 2, 6, 7, 3, 5), (1, 2, 7, 3, 5, 6), (1, 2, 3, 5, 6, 7)]
    space = S._Space(S.P2)
    for o in orders:
        mats, _, leaves, dead = A.derive_transform(S.P2, A.SEARCH_CANONICAL, orders=[list(o)])
        ref = S.greedy_canonical(S.P2, o, space=space)
        if ref is None:
            assert len(mats) == 0 and dead == 1 and leaves == 0
        else:
            assert len(mats) == 1 and np.array_equal(mats[0], ref) and leaves == 1


def test_topk_d2_matches_oracle(cuda):
    vec, idx, cos = A.search_topk(S.P2, 20)
    ref = S.topk_scan(S.P2, 20, chunk=100_000)
    for r in range(8):
        assert np.array_equal(idx[r], ref[r]["idx"])
        assert np.array_equal(vec[r], ref[r]["vec"])
        np.testing.assert_allclose(cos[r], ref[r]["cos"], rtol=0, atol=1e-15)


def test_topk_9pow8_and_tuples(cuda):
    """The 9^8 = 43,046,721-candidate space over P = {0, +-1, .., +-4}, top 256
    per row: lists, then the orthogonal 8-tuples at k = 64 (none) and 256."""
    vec, idx, cos = A.search_topk(S.P4, 256)
    ref = S.topk_scan(S.P4, 256)
    for r in range(8):
        assert np.array_equal(idx[r], ref[r]["idx"])
    for k in (64, 256):
        tups, n = A.orthogonal_tuples([vec[r][:k] for r in range(8)])
        rt, rn = ctuples.orthogonal_tuples([ref[r]["vec"][:k] for r in range(8)])
        assert n == rn
        assert np.array_equal(tups, rt)
    assert A.orthogonal_tuples([vec[r][:64] for r in range(8)])[1] == 0


def test_tuples_small_lists(cuda):
    rng = np.random.default_rng(3)
    for trial in range(5):
        lists = [rng.integers(-1, 2, size=(int(rng.integers(1, 9)), 8)) for _ in range(8)]
        tups, n = A.orthogonal_tuples(lists)
        py = S.orthogonal_tuples_py(lists)
        assert n == len(py)
        assert [tuple(t) for t in tups] == py


def test_search_argument_errors(cuda):
    with pytest.raises(A.AdctError):
        A.derive_transform([1, -1], A.SEARCH_CLOSURE)          # P without 0
    with pytest.raises(A.AdctError):
        A.derive_transform([0, 1, 1], A.SEARCH_CLOSURE)        # repeated entry
    with pytest.raises(A.AdctError):
        A.derive_transform(S.P1, A.SEARCH_CLOSURE, orders=[[1, 2, 3, 5, 6, 6]])
    with pytest.raises(A.AdctError):
        A.search_topk(S.P1, 0)


# ---------------------------------------------------------------- full orders and extended P

EXT_5 = [(0, 1, -1, 4, -4), (0, 1, -1, 8, -8)]
EXT_7 = [(0, 1, -1, 2, -2, 4, -4), (0, 1, -1, 2, -2, 8, -8), (0, 2, -2, 4, -4, 8, -8)]


def test_closure_d1_all_orders(cuda):
    """All 8! orders with no fixed rows (Sec. 3.5): matrices, leaves and dead paths."""
    mats, _, leaves, dead = A.derive_transform(S.P1, A.SEARCH_CLOSURE, fix_rows_1_5=False)
    ref, rleaves, rdead = S.closure(S.P1, orders=None, fixed=None)
    assert [_key(m) for m in mats] == [_key(m) for m in ref]
    assert (leaves, dead) == (rleaves, rdead) and leaves >= 40320


def test_canonical_d2_full_orders_sampled(cuda):
    """Per-order canonical results over random full orders of D2 (no fixed rows)."""
    rng = np.random.default_rng(11)
    space = S._Space(S.P2)
    for _ in range(30):
        o = [int(x) for x in rng.permutation(8)]
        mats, _, leaves, dead = A.derive_transform(S.P2, A.SEARCH_CANONICAL, orders=[o],
                                                   fix_rows_1_5=False)
        ref = S.greedy_canonical(S.P2, o, fixed=None, space=space)
        if ref is None:
            assert len(mats) == 0 and dead == 1
        else:
            assert len(mats) == 1 and _key(mats[0]) == _key(ref), o


@pytest.mark.parametrize("p", EXT_5)
def test_closure_extended_five_element_sets(cuda, p):
    """The extended entry sets of Sec. 4.1 with five elements: all 720 orders."""
    mats, _, leaves, dead = A.derive_transform(p, A.SEARCH_CLOSURE)
    ref, rleaves, rdead = S.closure(p)
    assert [_key(m) for m in mats] == [_key(m) for m in ref]
    assert (leaves, dead) == (rleaves, rdead)


@pytest.mark.parametrize("p", EXT_7)
def test_closure_extended_seven_element_sets_sampled(cuda, p):
    """The seven-element extended sets (7^8 = 5,764,801 vectors): closure over a
    sample of orders against the oracle."""
    rng = np.random.default_rng(10 * len(p) + abs(p[-1]) + abs(p[1]))
    orders = [tuple(int(x) for x in rng.permutation(list(S.FREE_ROWS))) for _ in range(6)]
    mats, _, leaves, dead = A.derive_transform(p, A.SEARCH_CLOSURE, orders=[list(o) for o in orders])
    ref, rleaves, rdead = S.closure(p, orders=orders)
    assert [_key(m) for m in mats] == [_key(m) for m in ref]
    assert (leaves, dead) == (rleaves, rdead)


def test_topk_extended_set_primitive(cuda):
    """Top-k over {0, +-1, +-2, +-8} with primitive vectors only (gcd 1 over
    entries up to 8)."""
    p = (0, 1, -1, 2, -2, 8, -8)
    vec, idx, cos = A.search_topk(p, 16, primitive=True)
    ref = S.topk_scan(p, 16, primitive=True)
    for r in range(8):
        assert np.array_equal(idx[r], ref[r]["idx"])
        assert np.array_equal(vec[r], ref[r]["vec"])
        np.testing.assert_allclose(cos[r], ref[r]["cos"], rtol=0, atol=1e-15)


def test_release_caches_then_search_again(cuda):
    """adct_release_caches frees the search buffers kept on the device (and the
    coding-gain sweep's); the next search allocates again and gives the same
    ranking; a second release finds nothing left."""
    vec, idx, cos = A.search_topk(S.P2, 20)
    A.coding_gain_sweep([M.T1.astype(np.float64) / np.sqrt((M.T1 ** 2).sum(1, keepdims=True))], [0.9])
    freed = A.release_caches()
    assert freed > 0
    assert A.release_caches() == 0
    vec2, idx2, cos2 = A.search_topk(S.P2, 20)
    assert np.array_equal(idx, idx2) and np.array_equal(vec, vec2) and np.array_equal(cos, cos2)
