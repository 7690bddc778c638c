"""FP64 brute-force Lloyd oracle (ctypes binding of ``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the GPU library.

The C source states what is computed and which passage of the paper each part
follows; this wrapper only marshals numpy arrays (float64 in, float32 inputs
are upcast exactly).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c11", "-Wall"]


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` next to it (gcc)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int
        lib.oracle_exact_sum.argtypes = [P, I64]
        lib.oracle_exact_sum.restype = ctypes.c_double
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_assign.argtypes = [P, I64, I32, P, I64, P, P]
        lib.oracle_update.argtypes = [P, I64, I32, P, I64, P, P, P]
        lib.oracle_lloyd.argtypes = [P, I64, I32, P, I64, I32, I32, P, P, P, P, P]
        lib.oracle_lloyd.restype = ctypes.c_int
        lib.oracle_distortion_fwd.argtypes = [P, P, I64, I64, I64, I32, P, P]
        lib.oracle_distortion_bwd.argtypes = [P, P, P, P, I64, I64, I64, I32, P, P]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def exact_sum(v) -> float:
    """Correctly rounded sum of a 1-D array of doubles."""
    v = _f64(v).ravel()
    return float(_load().oracle_exact_sum(_ptr(v), v.size))


def assign(x, c):
    """Lowest-index argmin of the canonical FP64 squared distance.

    Returns ``(a int32 [n], dmin float64 [n])``.
    """
    x, c = _f64(x), _f64(c)
    n, d = x.shape
    k = c.shape[0]
    a = np.empty(n, np.int32)
    dm = np.empty(n, np.float64)
    _load().oracle_assign(_ptr(x), n, d, _ptr(c), k, _ptr(a), _ptr(dm))
    return a, dm


def update(x, a, c_prev):
    """Centroids RN(exact cluster sum)/count; empty clusters keep ``c_prev``.

    Returns ``(c float64 [k,d], counts int64 [k])``.
    """
    x, c_prev = _f64(x), _f64(c_prev)
    a = np.ascontiguousarray(a, dtype=np.int32)
    n, d = x.shape
    k = c_prev.shape[0]
    c = np.empty_like(c_prev)
    cnt = np.empty(k, np.int64)
    _load().oracle_update(_ptr(x), n, d, _ptr(a), k, _ptr(c_prev), _ptr(c), _ptr(cnt))
    return c, cnt


def lloyd(x, c0, max_iter: int, stop_when_stable: bool = False, history: bool = True):
    """Run the Lloyd loop.

    Returns a dict with ``iters``, ``c`` (final), ``a`` (final) and, when
    ``history``, ``a_hist [T,n]``, ``c_hist [T,k,d]`` (C_t after iteration t)
    and ``sse [T]`` (objective of assignment a_t against C_{t-1}).
    """
    x, c0 = _f64(x), _f64(c0)
    n, d = x.shape
    k = c0.shape[0]
    a_hist = np.empty((max_iter, n), np.int32) if history else None
    c_hist = np.empty((max_iter, k, d), np.float64) if history else None
    sse = np.empty(max_iter, np.float64)
    c = np.empty_like(c0)
    a = np.empty(n, np.int32)
    t = _load().oracle_lloyd(_ptr(x), n, d, _ptr(c0), k, int(max_iter), int(bool(stop_when_stable)),
                             _ptr(a_hist), _ptr(c_hist), _ptr(sse), _ptr(c), _ptr(a))
    out = dict(iters=int(t), c=c, a=a, sse=sse[:t])
    if history:
        out.update(a_hist=a_hist[:t], c_hist=c_hist[:t])
    return out


def distortion_fwd(x, c):
    """Per-cloud loss RN(exact sum of D(x_i, c_a(i))) and the assignment.

    ``x [B,n,d]``, ``c [B,k,d]`` -> ``(a int32 [B,n], loss float64 [B])``.
    """
    x, c = _f64(x), _f64(c)
    B, n, d = x.shape
    k = c.shape[1]
    a = np.empty((B, n), np.int32)
    loss = np.empty(B, np.float64)
    _load().oracle_distortion_fwd(_ptr(x), _ptr(c), B, n, k, d, _ptr(a), _ptr(loss))
    return a, loss


def distortion_bwd(x, c, a, g):
    """Gradients of the per-cloud loss with the assignment held fixed.

    Returns ``(gx float64 [B,n,d], gc float64 [B,k,d])``.
    """
    x, c = _f64(x), _f64(c)
    a = np.ascontiguousarray(a, dtype=np.int32)
    g = _f64(g).ravel()
    B, n, d = x.shape
    k = c.shape[1]
    gx = np.empty_like(x)
    gc = np.empty_like(c)
    _load().oracle_distortion_bwd(_ptr(x), _ptr(c), _ptr(a), _ptr(g), B, n, k, d, _ptr(gx), _ptr(gc))
    return gx, gc
