"""ctypes loader for oracle.c (TEST INFRASTRUCTURE ONLY).

``build()`` compiles ``oracle.c`` with gcc (-O2 -fopenmp, plain C, fp64) into
``oracle/liboracle.so``.  ``load()`` builds on first use when the library is absent.
All wrappers take float64 NumPy arrays and return float64 / int64 results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_dtw_pow.restype = ctypes.c_double
    lib.orc_dtw_pow.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_dtw_pow_many.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
    lib.orc_lb_many.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.orc_envelope.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.orc_nn_bruteforce.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, _ip, _dp]
    lib.orc_nn_sequential_many.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, _ip, _dp, _ip]
    _lib = lib
    return lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def _p(p) -> int:
    return 0 if p == np.inf else int(p)


def num_threads() -> int:
    return int(load().orc_num_threads())


def set_num_threads(threads: int) -> None:
    """Threads used by the OpenMP loops of the following calls."""
    load().orc_set_num_threads(int(threads))


def envelope(y, w):
    y = _c(y)
    n = y.size
    U, L = np.empty(n), np.empty(n)
    load().orc_envelope(_ptr(y), n, int(w), _ptr(U), _ptr(L))
    return U, L


def dtw_pow(x, y, w, p) -> float:
    x, y = _c(x), _c(y)
    return float(load().orc_dtw_pow(_ptr(x), _ptr(y), x.size, int(w), _p(p)))


def dtw_pow_many(X, y, w, p) -> np.ndarray:
    X, y = _c(X), _c(y)
    out = np.empty(X.shape[0])
    load().orc_dtw_pow_many(_ptr(X), X.shape[0], _ptr(y), X.shape[1], int(w), _p(p), _ptr(out))
    return out


def lb_many(X, y, w, p):
    """(LB_Keogh^p, LB_Improved^p) of every row of X against y."""
    X, y = _c(X), _c(y)
    s1, s2 = np.empty(X.shape[0]), np.empty(X.shape[0])
    load().orc_lb_many(_ptr(X), X.shape[0], _ptr(y), X.shape[1], int(w), _p(p), _ptr(s1), _ptr(s2))
    return s1, s2


def nn_bruteforce(DB, Qs, w, p, k=1):
    """(idx [nq][k], pow distances [nq][k]) by brute force."""
    DB, Qs = _c(DB), _c(np.atleast_2d(Qs))
    nq, n = Qs.shape
    idx = np.empty((nq, k), dtype=np.int64)
    dist = np.empty((nq, k))
    load().orc_nn_bruteforce(_ptr(DB), DB.shape[0], _ptr(Qs), nq, n, int(w), _p(p), int(k), _ptr(idx, _ip),
                             _ptr(dist))
    return idx, dist


def nn_sequential(DB, Qs, w, p, improved: bool):
    """Algorithm 2 / 3 per query: (idx [nq], pow distance [nq], counters [nq][3])."""
    DB, Qs = _c(DB), _c(np.atleast_2d(Qs))
    nq, n = Qs.shape
    idx = np.empty(nq, dtype=np.int64)
    dist = np.empty(nq)
    cnt = np.empty((nq, 3), dtype=np.int64)
    load().orc_nn_sequential_many(_ptr(DB), DB.shape[0], _ptr(Qs), nq, n, int(w), _p(p), int(bool(improved)),
                                  _ptr(idx, _ip), _ptr(dist), _ptr(cnt, _ip))
    return idx, dist, cnt
