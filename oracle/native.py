"""Loader for the oracle's C helper (``crsum.c``): correctly rounded FP64 sums.

Test infrastructure only.  Nothing in the product package imports this module;
only ``tests/``, the smoke check and the benchmark's CPU-baseline leg do.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crsum.c")
_LIB = os.path.join(_HERE, "_crsum.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile crsum.c with gcc (IEEE doubles: no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.cr_sum.restype = ctypes.c_double
        L.cr_sum.argtypes = [dp, ctypes.c_int64]
        L.cr_dot.restype = ctypes.c_double
        L.cr_dot.argtypes = [dp, dp, ctypes.c_int64]
        L.cr_csr_rowsum.restype = None
        L.cr_csr_rowsum.argtypes = [ctypes.c_int64, ip, ip, dp, dp, ctypes.c_int32, dp,
                                    ctypes.POINTER(dp), dp]
        L.cr_rows_comb.restype = None
        L.cr_rows_comb.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, dp, dp, dp]
        L.cr_gram.restype = None
        L.cr_gram.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, dp]
        L.ord_gram.restype = None
        L.ord_gram.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, ctypes.c_int64, dp]
        L.cr_num_threads.restype = ctypes.c_int
        L.cr_num_threads.argtypes = []
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def cr_sum(t) -> float:
    t = _f64(t)
    return float(lib().cr_sum(_dp(t), t.size))


def cr_dot(x, y) -> float:
    x = _f64(x)
    y = _f64(y)
    assert x.shape == y.shape
    return float(lib().cr_dot(_dp(x), _dp(y), x.size))


def cr_csr_rowsum(rowptr, col, val, u, extra=()) -> np.ndarray:
    """out[i] = RN(sum_k val[k] u[col[k]] + sum_e c_e v_e[i]) for extra = [(c_e, v_e)]."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = _f64(val)
    u = _f64(u)
    n = rowptr.size - 1
    out = np.empty(n, dtype=np.float64)
    coefs = np.array([float(c) for c, _ in extra], dtype=np.float64)
    vecs = [_f64(v) for _, v in extra]
    for v in vecs:
        assert v.size == n
    VP = ctypes.POINTER(ctypes.c_double) * max(1, len(vecs))
    vp = VP(*[_dp(v) for v in vecs]) if vecs else VP()
    lib().cr_csr_rowsum(n, _ip(rowptr), _ip(col), _dp(val), _dp(u), len(vecs),
                        _dp(coefs) if len(coefs) else None, vp, _dp(out))
    return out


def cr_rows_comb(cols, coef, base=None) -> np.ndarray:
    """out[i] = RN(base[i] + sum_a cols[a][i] * coef[a])."""
    Y = np.ascontiguousarray(np.stack([_f64(c) for c in cols]), dtype=np.float64)
    d, n = Y.shape
    c = _f64(coef)
    assert c.size == d
    out = np.empty(n, dtype=np.float64)
    b = _f64(base) if base is not None else None
    lib().cr_rows_comb(n, d, _dp(Y), n, _dp(c), _dp(b) if b is not None else None, _dp(out))
    return out


def cr_gram(cols) -> np.ndarray:
    """G[a,b] = RN(sum_i cols[a][i] cols[b][i]) for all a, b."""
    Y = np.ascontiguousarray(np.stack([_f64(c) for c in cols]), dtype=np.float64)
    d, n = Y.shape
    G = np.empty((d, d), dtype=np.float64)
    lib().cr_gram(n, d, _dp(Y), n, _dp(G))
    return G


def ord_gram(cols) -> np.ndarray:
    """G = Y^T Y in the stated order: fma chains over 1024-row groups, pairwise
    summation of the group partials (see crsum.c)."""
    Y = np.ascontiguousarray(np.stack([_f64(c) for c in cols]), dtype=np.float64)
    d, n = Y.shape
    G = np.empty((d, d), dtype=np.float64)
    lib().ord_gram(n, d, _dp(Y), n, _dp(G))
    return G


def num_threads() -> int:
    return int(lib().cr_num_threads())


def threads_env() -> int:
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else num_threads()
