"""ctypes binding of oracle/rowpar.c: the row-parallel (OpenMP, all host
cores) FP64 product of a CSR matrix, for the CPU baseline.

TEST INFRASTRUCTURE ONLY (bench.py's CPU baseline and its test)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rowpar.c")
_LIB = os.path.join(_HERE, "librowpar.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.oracle_rowpar_spmv.argtypes = [ctypes.c_int64, P, P, P, P, P]
        L.oracle_rowpar_spmv.restype = None
        L.oracle_rowpar_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    return int(_load().oracle_rowpar_threads())


def spmv(A, x):
    """out = A @ x for a scipy CSR matrix A (float64 data), rows in parallel."""
    L = _load()
    rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = np.ascontiguousarray(A.data, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(A.shape[0])
    L.oracle_rowpar_spmv(A.shape[0], rp.ctypes.data, col.ctypes.data, val.ctypes.data, xx.ctypes.data,
                         out.ctypes.data)
    return out
