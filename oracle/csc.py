"""ctypes wrapper of the plain-C Slater-Condon sigma (oracle; test infrastructure only).

`build()` compiles oracle/sc_sigma.c with gcc (OpenMP) into oracle/_sc_sigma.so.
All arrays crossing the boundary are complex128 (real inputs are promoted).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_sigma.c")
_LIB = os.path.join(_HERE, "_sc_sigma.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_sigma.argtypes = [ctypes.c_int, I64, P, P, P, ctypes.c_double, P, P, ctypes.c_int]
        lib.oracle_sigma_rows.argtypes = [ctypes.c_int, I64, P, P, P, ctypes.c_double, P, P, I64, P,
                                          ctypes.c_int]
        lib.oracle_h_row.argtypes = [ctypes.c_int, I64, P, P, P, ctypes.c_double, I64, P, I64]
        lib.oracle_h_row.restype = I64
        lib.oracle_diag.argtypes = [ctypes.c_int, I64, P, P, P, ctypes.c_double, P, ctypes.c_int]
        lib.oracle_h_row_window.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, ctypes.c_double,
                                            ctypes.c_uint64, P, P, I64]
        lib.oracle_h_row_window.restype = I64
        _lib = lib
    return _lib


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _threads(n):
    return int(n) if n else (os.cpu_count() or 1)


def sigma(dets, h, g, c, e_core=0.0, nthreads=0):
    """sigma = P H P c over the sorted determinant list `dets` (uint64)."""
    lib = _load()
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    h, g, c = _c128(h), _c128(g), _c128(c)
    out = np.zeros(len(dets), dtype=np.complex128)
    lib.oracle_sigma(h.shape[0], len(dets), _ptr(dets), _ptr(h), _ptr(g), float(e_core), _ptr(c),
                     _ptr(out), _threads(nthreads))
    return out


def sigma_rows(dets, h, g, c, rows, e_core=0.0, nthreads=0):
    """sigma_L for the selected row indices only."""
    lib = _load()
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    h, g, c = _c128(h), _c128(g), _c128(c)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(len(rows), dtype=np.complex128)
    lib.oracle_sigma_rows(h.shape[0], len(dets), _ptr(dets), _ptr(h), _ptr(g), float(e_core), _ptr(c),
                          _ptr(rows), len(rows), _ptr(out), _threads(nthreads))
    return out


def h_row(dets, h, g, row, e_core=0.0):
    """Nonzero couplings of one row: (column indices, values)."""
    lib = _load()
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    h, g = _c128(h), _c128(g)
    cap = 1 << 16
    while True:
        buf = np.zeros(3 * cap)
        n = lib.oracle_h_row(h.shape[0], len(dets), _ptr(dets), _ptr(h), _ptr(g), float(e_core), int(row),
                             _ptr(buf), cap)
        if n <= cap:
            break
        cap = int(n)
    buf = buf[:3 * n].reshape(n, 3)
    return buf[:, 0].astype(np.int64), buf[:, 1] + 1j * buf[:, 2]


def h_row_window(sub, lo, hi, h, g, bits, e_core=0.0):
    """Row of P H P for determinant `bits` of the windowed space (subspace
    sizes sub, windows [lo, hi]) without a determinant list: (column bit
    strings, values), the diagonal first."""
    lib = _load()
    h, g = _c128(h), _c128(g)
    K = len(sub)
    lo = list(lo) if lo is not None else [0] * K
    hi = list(hi) if hi is not None else list(sub)
    arr = lambda x: np.ascontiguousarray(x, dtype=np.int32)
    sub_a, lo_a, hi_a = arr(sub), arr(lo), arr(hi)
    cap = 1 << 16
    while True:
        ob = np.zeros(cap, dtype=np.uint64)
        ov = np.zeros(2 * cap)
        n = lib.oracle_h_row_window(h.shape[0], K, _ptr(sub_a), _ptr(lo_a), _ptr(hi_a), _ptr(h), _ptr(g),
                                    float(e_core), ctypes.c_uint64(int(bits)), _ptr(ob), _ptr(ov), cap)
        if n <= cap:
            break
        cap = int(n)
    return ob[:n], ov[0:2 * n:2] + 1j * ov[1:2 * n:2]


def diag(dets, h, g, e_core=0.0, nthreads=0):
    lib = _load()
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    h, g = _c128(h), _c128(g)
    out = np.zeros(len(dets))
    lib.oracle_diag(h.shape[0], len(dets), _ptr(dets), _ptr(h), _ptr(g), float(e_core), _ptr(out),
                    _threads(nthreads))
    return out
