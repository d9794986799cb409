"""The no-allocation coding-gain sweep (for callers that cannot allocate device
memory) against the allocating entry point, through the C ABI: two calls in a
row, the second with fewer matrices and correlations, each bit-identical to
adct_coding_gain_sweep (same kernel, same inputs)."""

import ctypes

import numpy as np
import pytest

import paper_1808_02950_amd as A
from oracle import matrices as M

pytestmark = pytest.mark.gpu


def _c_hats(names):
    return np.stack([M.approx_matrix(M.TRANSFORMS[n]) if n != "DCT" else M.dct_matrix() for n in names])


def _call_noalloc(c, rho):
    c = np.ascontiguousarray(c.reshape(-1, 64))
    rho = np.ascontiguousarray(rho)
    out = np.full((c.shape[0], rho.shape[0]), np.nan)
    st = A.lib().adct_coding_gain_sweep_noalloc(c.ctypes.data, c.shape[0], rho.ctypes.data, rho.shape[0],
                                                out.ctypes.data, None)
    assert st == 0, A.lib().adct_last_error()
    return out


def test_noalloc_matches_allocating_sweep_twice(cuda):
    big_c = _c_hats(["DCT", "T1", "T2", "LO", "T6", "RDCT", "T4"])
    big_rho = np.linspace(0.0, 0.999, 2000)
    small_c = _c_hats(["T1", "LO"])
    small_rho = np.array([0.95, 0.5, 0.1])
    first = _call_noalloc(big_c, big_rho)
    want = A.coding_gain_sweep(big_c, big_rho)
    assert np.array_equal(first, want)
    second = _call_noalloc(small_c, small_rho)
    want2 = A.coding_gain_sweep(small_c, small_rho)
    assert np.array_equal(second, want2)
    assert np.all(np.isfinite(second))
    # the measures table's C_g* differences against the DCT at rho = 0.95
    assert abs((want[1, np.argmin(np.abs(big_rho - 0.95))] - want[0, np.argmin(np.abs(big_rho - 0.95))])) < 0.3


def test_noalloc_limit_and_errors(cuda):
    c = _c_hats(["T1"])
    rho = np.zeros(262145 - 64)                      # 64 + n_rho + n_rho > 2^18
    out = np.zeros(rho.shape[0])
    st = A.lib().adct_coding_gain_sweep_noalloc(c.ctypes.data, 1, rho.ctypes.data, rho.shape[0],
                                                out.ctypes.data, None)
    assert st == -3
    assert b"262,144" in A.lib().adct_last_error()
    # the largest sweep that fits still works and equals the allocating one
    n_rho = (262144 - 64) // 2
    rho = np.linspace(0.0, 0.99, n_rho)
    assert np.array_equal(_call_noalloc(c, rho), A.coding_gain_sweep(c, rho))
