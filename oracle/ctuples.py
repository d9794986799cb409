"""ctypes loader for the plain-C orthogonal-tuple enumeration (`tuples.c`).

TEST INFRASTRUCTURE: see the package docstring.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tuples.c")
_LIB = os.path.join(_HERE, "libtuples.so")
_handle = None


def build(force: bool = True) -> str:
    """Compile tuples.c with gcc into oracle/libtuples.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        h = ctypes.CDLL(_LIB)
        h.oracle_orthogonal_tuples.restype = ctypes.c_int64
        h.oracle_orthogonal_tuples.argtypes = [
            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
            ctypes.c_void_p, ctypes.c_int64]
        _handle = h
    return _handle


def orthogonal_tuples(lists: list[np.ndarray], cap: int = 1 << 20):
    """Returns (tuples (n, 8) int32 of list positions, total count)."""
    arrs = [np.ascontiguousarray(np.asarray(l, dtype=np.int8).reshape(-1, 8)) for l in lists]
    if len(arrs) != 8:
        raise ValueError("need 8 lists")
    ptrs = (ctypes.c_void_p * 8)(*[a.ctypes.data if a.size else None for a in arrs])
    lens = (ctypes.c_int * 8)(*[a.shape[0] for a in arrs])
    out = np.zeros((max(cap, 1), 8), dtype=np.int32)
    n = _lib().oracle_orthogonal_tuples(ptrs, lens, out.ctypes.data, cap)
    if n < 0:
        raise RuntimeError("orthogonal tuple enumeration failed")
    return out[:min(n, cap)], int(n)
