"""ctypes wrapper of the plain C Bareiss determinant (oracle/bareiss.c).

TEST INFRASTRUCTURE ONLY (part of the oracle).  ``build_bareiss_c`` compiles
the C file with gcc into ``oracle/_bareiss.so``; ``det_bareiss_c`` returns
det(A) as a Python int.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bareiss.c")
_LIB = os.path.join(_HERE, "_bareiss.so")
_handle = None


def build_bareiss_c(force: bool = True) -> str:
    """Compile oracle/bareiss.c (gcc -O2 -fopenmp) into oracle/_bareiss.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB):
            build_bareiss_c(force=False)
        h = ctypes.CDLL(_LIB)
        h.oracle_bareiss_det.restype = ctypes.c_int
        h.oracle_bareiss_det.argtypes = [
            ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(ctypes.c_uint32), ctypes.c_int,
            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        _handle = h
    return _handle


def det_bareiss_c(A, threads: int = 0) -> int:
    """Exact det(A) (A: n x n integers with |a_ij| < 2^63) by the C Bareiss.
    threads = 0 lets OpenMP choose."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    n = A.shape[0]
    if A.ndim != 2 or A.shape[1] != n:
        raise ValueError("square matrix expected")
    lib = _lib()
    cap = max(4, n * 4 + 8)
    while True:
        mag = (ctypes.c_uint32 * cap)()
        out_len = ctypes.c_int(0)
        out_sign = ctypes.c_int(0)
        st = lib.oracle_bareiss_det(
            A.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, threads, mag, cap,
            ctypes.byref(out_len), ctypes.byref(out_sign))
        if st == 1:
            cap = out_len.value
            continue
        if st != 0:
            raise RuntimeError(f"oracle_bareiss_det failed with status {st}")
        v = 0
        for i in range(out_len.value - 1, -1, -1):
            v = (v << 32) | mag[i]
        return out_sign.value * v
