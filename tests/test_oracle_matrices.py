"""Pins of the oracle's matrices and measures against what the paper prints."""

import json
import math
import os

import numpy as np
import pytest
from scipy.fft import dct as scipy_dct

from oracle import matrices as M
from oracle import measures as Me

GOLD = os.path.join(os.path.dirname(__file__), "golden")

NAMED = {"T1": M.T1, "T2": M.T2, "LO": M.T_LO_X2, "SDCT": M.t_sdct(), "RDCT": M.T_RDCT,
         "BAS2008B": M.T_BAS2008B, "T4": M.T4, "T6": M.T6}


def test_dct_closed_form_matches_library_dct():
    # orthonormal DCT-II from scipy is an independent definition of the same matrix
    ref = scipy_dct(np.eye(8), type=2, norm="ortho", axis=0)
    np.testing.assert_allclose(M.dct_matrix(), ref, atol=1e-15)


def test_printed_dct_is_twice_orthonormal():
    np.testing.assert_allclose(M.dct_matrix_as_printed(), 2.0 * M.dct_matrix(), atol=1e-15)
    c = M.dct_matrix()
    np.testing.assert_allclose(c @ c.T, np.eye(8), atol=1e-15)


def test_s1_diagonal_as_printed():
    gold = json.load(open(os.path.join(GOLD, "search_results.json")))
    assert list(M.row_norms2(M.T1)) == gold["S1_diag_squared_inverse"]
    assert list(M.row_norms2(M.T2)) == gold["S1_diag_squared_inverse"]
    np.testing.assert_allclose(M.scale_diag(M.T1), 1 / np.sqrt(gold["S1_diag_squared_inverse"]))


@pytest.mark.parametrize("name", ["T1", "T2", "LO", "T6", "RDCT", "T4"])
def test_orthogonal_matrices(name):
    t = NAMED[name]
    assert M.is_orthogonal_rows(t)
    c_hat = M.approx_matrix(t)
    np.testing.assert_allclose(c_hat @ c_hat.T, np.eye(8), atol=1e-15)
    # rows 1 and 5 are the trivial +-1 rows up to a positive factor (Sec. 4.1)
    assert len(set(t[0])) == 1 and t[0][0] > 0
    assert np.all(np.sign(t[4]) == [1, -1, -1, 1, 1, -1, -1, 1])
    # for orthogonal T the row normalisation equals the literal matrix square root of Eq. (2)
    np.testing.assert_allclose(M.polar_factor(t), c_hat, atol=1e-12)


@pytest.mark.parametrize("name", ["SDCT", "BAS2008B"])
def test_non_orthogonal_matrices(name):
    assert not M.is_orthogonal_rows(NAMED[name])


def test_scale_reading_row_normalisation():
    # BAS-2008b's printed error energy is reproduced only by the row-normalised S
    gold = json.load(open(os.path.join(GOLD, "measures_table.json")))["rows"]["BAS2008B"]
    eps_rows = Me.total_error_energy(M.approx_matrix(M.T_BAS2008B))
    eps_polar = Me.total_error_energy(M.polar_factor(M.T_BAS2008B))
    assert round(eps_rows, 4) == gold["eps"]
    assert abs(eps_polar - gold["eps"]) > 0.5


@pytest.mark.parametrize("name", list(NAMED) + ["DCT"])
def test_measures_table(name):
    gold = json.load(open(os.path.join(GOLD, "measures_table.json")))["rows"][name]
    got = Me.dct_measures() if name == "DCT" else Me.measures(NAMED[name])
    for key in ("eps", "mse", "cg_star", "eta"):
        assert abs(got[key] - gold[key]) <= 0.51e-4, (key, got[key], gold[key])


@pytest.mark.parametrize("name", list(NAMED) + ["DCT"])
def test_circular_table(name):
    gold = json.load(open(os.path.join(GOLD, "circular_table.json")))["rows"][name]
    got = Me.circular_stats(M.dct_matrix() if name == "DCT" else NAMED[name])
    assert abs(got["theta_bar_deg"] - gold["theta_bar_deg"]) < 0.01
    assert abs(got["V"] - gold["V"]) <= 0.51e-4
    assert abs(got["D_mod"] - gold["D_mod"]) <= 0.51e-4


def test_error_energy_is_sum_of_row_angles():
    # for unit rows, ||c_k - c_hat_k||^2 = 2 (1 - cos angle_k): eps = pi sum 2(1 - cos)
    for t in (M.T1, M.T6, M.T_RDCT):
        c_hat = M.approx_matrix(t)
        cos = np.sum(c_hat * M.dct_matrix(), axis=1)
        assert abs(Me.total_error_energy(c_hat) - math.pi * np.sum(2 * (1 - cos))) < 1e-12


def test_orthogonal_coding_gain_agrees_with_unified():
    for t in (M.T1, M.T6, M.T4):
        c_hat = M.approx_matrix(t)
        assert abs(Me.coding_gain(c_hat) - Me.unified_coding_gain(c_hat)) < 1e-9
