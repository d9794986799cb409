"""Pins of the fast algorithm for T1 (Sec. 5.1)."""

import json
import os

import numpy as np

from oracle import matrices as M
from oracle import sfg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_factorisation_is_t1():
    assert np.array_equal(np.array(sfg.factor_product(), dtype=np.int64), M.T1)


def test_sfg_matches_matrix_on_random_vectors():
    # the paper checks its FPGA design against 100,000 random 8-point vectors (Sec. 5.2)
    rng = np.random.default_rng(2018)
    x = rng.integers(-(1 << 20), 1 << 20, size=(100_000, 8))
    y = np.stack(sfg.t1_sfg([x[:, k] for k in range(8)]), axis=1)
    assert np.array_equal(y, x @ M.T1.T)
    basis = np.eye(8, dtype=np.int64)
    yb = np.stack(sfg.t1_sfg([basis[:, k] for k in range(8)]), axis=1)
    assert np.array_equal(yb, M.T1.T)   # column k of T1 for basis vector e_k


def test_operation_counts():
    gold = json.load(open(os.path.join(GOLD, "cost_table.json")))
    assert sfg.sfg_cost() == (gold["T1_fast"]["adds"], gold["T1_fast"]["shifts"])
    assert sfg.direct_cost(M.T1) == (gold["T1_direct"]["adds"], gold["T1_direct"]["shifts"])


def test_int16_range_of_two_passes():
    # interval propagation of [0, 255] through row then column pass: T1's
    # integer stage fits int16, the doubled LO matrix does not
    def bound(t):
        t = np.asarray(t, dtype=np.int64)
        k = np.einsum("ku,lv->kluv", t, t)
        return 255 * max(np.clip(k, 0, None).sum(axis=(2, 3)).max(),
                         np.clip(-k, 0, None).sum(axis=(2, 3)).max())
    assert bound(M.T1) == 18360 < 32768
    assert bound(M.T_LO_X2) == 65280 > 32767
