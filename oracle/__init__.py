"""CPU FP64 oracle of standard K-means -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, the smoke check in `__graft_entry__` and the CPU-baseline leg
of `bench.py` may import this package.  The GPU library never does, and the
two share no code: this side is plain C (`lloyd64.c`) driven through ctypes.

What it computes is Lloyd's algorithm in FP64, direct form, with ties going
to the lowest centroid index and empty clusters keeping their centroid
(paper, Abstract and Sections 1-2: the filtered method must return exactly
what "standard K-means" returns; the paper gives no formula, so the
textbook definition is used).

Pins (tests/test_oracle.py) tie it to things other than itself: a worked
1-D example derived by hand, brute-force enumeration of all labelings on
tiny inputs, the K=1 global mean, K=N with distinct points, constructed
exact ties, an empty cluster, SSE monotonicity and an independent library
implementation of Lloyd's algorithm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lloyd64.c")
_LIB = os.path.join(_HERE, "liblloyd64.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force=False):
    """Compile lloyd64.c with gcc -O2 -fopenmp into liblloyd64.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.kpo_threads.argtypes = [ctypes.c_int]
        lib.kpo_threads.restype = ctypes.c_int
        lib.kpo_assign.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _f64p, ctypes.c_int,
                                   _i32p, vp, vp, ctypes.c_int]
        lib.kpo_assign.restype = None
        lib.kpo_dist2_to.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _f64p, _i32p, _f64p,
                                     ctypes.c_int]
        lib.kpo_dist2_to.restype = None
        lib.kpo_update.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _i32p, ctypes.c_int,
                                   _f64p, _f64p, _i64p, ctypes.c_int]
        lib.kpo_update.restype = None
        lib.kpo_sse.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _f64p, _i32p, ctypes.c_int]
        lib.kpo_sse.restype = ctypes.c_double
        lib.kpo_lloyd.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _f64p, ctypes.c_int,
                                  ctypes.c_int, vp, vp, vp, vp, _f64p, ctypes.c_int]
        lib.kpo_lloyd.restype = None
        _lib = lib
    return _lib


def _x(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be (n, d)")
    return X


def _c(C, d):
    C = np.ascontiguousarray(C, dtype=np.float64)
    if C.ndim != 2 or C.shape[1] != d:
        raise ValueError("C must be (k, d)")
    return C


def threads(n=0):
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return _load().kpo_threads(int(n))


def assign(X, C, *, second=False, nthreads=0):
    """Nearest centroid per point: (labels int32, d1^2 float64[, d2^2]).

    FP64 direct form; exact ties go to the lowest centroid index.
    """
    X = _x(X)
    C = _c(C, X.shape[1])
    n = X.shape[0]
    lab = np.empty(n, np.int32)
    d1 = np.empty(n, np.float64)
    d2 = np.empty(n, np.float64) if second else None
    _load().kpo_assign(X, n, X.shape[1], C, C.shape[0], lab, d1.ctypes.data,
                       d2.ctypes.data if second else None, int(nthreads))
    return (lab, d1, d2) if second else (lab, d1)


def dist2_to(X, C, labels, *, nthreads=0):
    """FP64 squared distance of each point to the centroid `labels` names."""
    X = _x(X)
    C = _c(C, X.shape[1])
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    if labels.shape != (X.shape[0],) or (labels.size and (labels.min() < 0 or labels.max() >= C.shape[0])):
        raise ValueError("labels out of range")
    out = np.empty(X.shape[0], np.float64)
    _load().kpo_dist2_to(X, X.shape[0], X.shape[1], C, labels, out, int(nthreads))
    return out


def update(X, labels, C_prev, *, nthreads=0):
    """FP64 means per centroid; an empty centroid keeps C_prev. -> (C, counts)."""
    X = _x(X)
    C_prev = _c(C_prev, X.shape[1])
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    k = C_prev.shape[0]
    if labels.shape != (X.shape[0],) or (labels.size and (labels.min() < 0 or labels.max() >= k)):
        raise ValueError("labels out of range")
    Cn = np.empty_like(C_prev)
    cnt = np.empty(k, np.int64)
    _load().kpo_update(X, X.shape[0], X.shape[1], labels, k, C_prev, Cn, cnt, int(nthreads))
    return Cn, cnt


def sse(X, C, labels, *, nthreads=0):
    """Sum over points of the squared FP64 distance to the labelled centroid."""
    X = _x(X)
    C = _c(C, X.shape[1])
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    return float(_load().kpo_sse(X, X.shape[0], X.shape[1], C, labels, int(nthreads)))


def lloyd(X, C0, iters, *, keep_labels=True, keep_centroids=True, nthreads=0):
    """Run `iters` Lloyd iterations from C0 in FP64.

    Returns a dict with per-iteration `labels` (T, n), `centroids` (T, k, d)
    -- the centroids after each iteration -- `sse_assign` and `sse_update`
    (T,), and `final` (k, d).
    """
    X = _x(X)
    C0 = _c(C0, X.shape[1])
    n, d = X.shape
    k = C0.shape[0]
    T = int(iters)
    lab = np.empty((T, n), np.int32) if keep_labels else None
    Cs = np.empty((T, k, d), np.float64) if keep_centroids else None
    sa = np.empty(T, np.float64)
    su = np.empty(T, np.float64)
    fin = np.empty((k, d), np.float64)
    _load().kpo_lloyd(X, n, d, C0, k, T,
                      lab.ctypes.data if lab is not None else None,
                      Cs.ctypes.data if Cs is not None else None,
                      sa.ctypes.data, su.ctypes.data, fin, int(nthreads))
    return dict(labels=lab, centroids=Cs, sse_assign=sa, sse_update=su, final=fin)
