"""ctypes access to the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bt_oracle.c")
_LIB = os.path.join(_HERE, "libbt_oracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -fopenmp into oracle/libbt_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-Wall", "-Wextra", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    """Open an oracle build (the default one, or a variant compiled by a test)."""
    L = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.bto_support.argtypes = [i32, i32, i64, p, p, p, p, p, ctypes.c_int, ctypes.c_int]
    L.bto_support.restype = ctypes.c_int
    L.bto_bitruss.argtypes = [i32, i32, i64, p, p, p, p, p, ctypes.c_int]
    L.bto_bitruss.restype = ctypes.c_int
    L.bto_edge_support.argtypes = [i32, p, p, p, p, i64]
    L.bto_edge_support.restype = i64
    L.bto_max_threads.restype = ctypes.c_int
    return L


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load_library(_LIB)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32))


def max_threads() -> int:
    return int(_load().bto_max_threads())


def support(n_upper, n_lower, row_ptr, col, orientation: int = 0, threads: int = 0, lib=None):
    """Per-edge butterfly supports (int64[m]) and the butterfly total two ways.

    Returns (sup, butterflies_from_sum_over_4, butterflies_from_pairs).
    orientation: 0 automatic, 1 start from the upper layer, 2 from the lower.
    """
    rp, c = _csr(row_ptr, col)
    m = c.shape[0]
    sup = np.zeros(m, dtype=np.int64)
    b = ctypes.c_int64(0)
    pr = ctypes.c_int64(0)
    rc = (lib or _load()).bto_support(int(n_upper), int(n_lower), m, _ptr(rp), _ptr(c), _ptr(sup),
                             ctypes.byref(b), ctypes.byref(pr), int(orientation), int(threads))
    if rc != 0:
        raise MemoryError("oracle support failed")
    return sup, int(b.value), int(pr.value)


def bitruss(n_upper, n_lower, row_ptr, col, sup=None, threads: int = 0, lib=None):
    """Bitruss number of every edge (int64[m]) and peel statistics.

    Returns (phi, stats) with stats = dict(levels, rounds, destroyed, max_phi);
    `destroyed` counts butterflies, each destroyed exactly once.
    """
    rp, c = _csr(row_ptr, col)
    m = c.shape[0]
    phi = np.zeros(m, dtype=np.int64)
    st = np.zeros(4, dtype=np.int64)
    sp = None
    if sup is not None:
        sup = np.ascontiguousarray(sup, dtype=np.int64)
        sp = _ptr(sup)
    rc = (lib or _load()).bto_bitruss(int(n_upper), int(n_lower), m, _ptr(rp), _ptr(c), sp,
                             _ptr(phi), _ptr(st), int(threads))
    if rc != 0:
        raise MemoryError("oracle bitruss failed")
    return phi, dict(levels=int(st[0]), rounds=int(st[1]), destroyed=int(st[2]),
                     max_phi=int(st[3]))


class _Transpose:
    def __init__(self, n_upper, n_lower, row_ptr, col):
        self.row_ptr, self.col = _csr(row_ptr, col)
        u = np.repeat(np.arange(n_upper, dtype=np.int32), np.diff(self.row_ptr))
        order = np.lexsort((u, self.col))
        self.ladj = np.ascontiguousarray(u[order], dtype=np.int32)
        self.lptr = np.zeros(n_lower + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.col, minlength=n_lower), out=self.lptr[1:])
        self.n_upper = n_upper


def edge_support(n_upper, n_lower, row_ptr, col, edges):
    """Supports of selected edge ids, each counted from the definition alone."""
    t = _Transpose(n_upper, n_lower, row_ptr, col)
    L = _load()
    return np.array([L.bto_edge_support(t.n_upper, _ptr(t.row_ptr), _ptr(t.col),
                                        _ptr(t.lptr), _ptr(t.ladj), int(e))
                     for e in np.asarray(edges).ravel()], dtype=np.int64)
