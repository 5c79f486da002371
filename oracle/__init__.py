"""TEST INFRASTRUCTURE ONLY: the CPU oracle for range-discord search.

``merlin.c`` is a plain serial FP64 implementation of MERLIN driving DRAG
(Sec. 2.2, Alg. 1-2) and ``bruteforce.py`` evaluates the discord definition
directly (Sec. 2.1).  Neither shares code with the GPU library.  Only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.

The C part is compiled by ``oracle.build_lib()`` (called from
``__graft_entry__.build()``) into ``oracle/liboracle.so`` (serial) and, from
the same source with ``-fopenmp``, ``oracle/liboracle_omp.so``, whose DRAG
phases split their inner candidate loop over threads with identical results;
``merlin(..., threads=t)`` uses the latter for the largest workloads.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "merlin.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build_lib(force: bool = True) -> str:
    """Compile merlin.c with gcc (plain -O2, no fast-math) into liboracle.so,
    and once more with -fopenmp into liboracle_omp.so."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                                   *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


def _load(path):
    if not os.path.exists(path):
        build_lib(force=False)
    L = ctypes.CDLL(path)
    L.oracle_threads.argtypes = [ctypes.c_int]
    L.oracle_threads.restype = ctypes.c_int
    return L


def lib(threads: int | None = None):
    """The serial library, or the OpenMP one set to ``threads`` threads."""
    global _lib, _lib_omp
    if threads is not None:
        if _lib_omp is None:
            _lib_omp = _bind(_load(_LIB_OMP))
        _lib_omp.oracle_threads(int(threads))
        return _lib_omp
    if _lib is None:
        _lib = _bind(_load(_LIB))
    return _lib


def _bind(L):
    L.oracle_window_stats.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, _f64p, _f64p]
    L.oracle_window_stats.restype = None
    L.oracle_drag.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                              _i64p, _f64p, _i64p, _i64p, _u64p]
    L.oracle_drag.restype = ctypes.c_int
    L.oracle_nn_row.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                _f64p, _i64p]
    L.oracle_nn_row.restype = ctypes.c_int
    L.oracle_merlin.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p,
                                _u64p]
    L.oracle_merlin.restype = ctypes.c_int
    L.oracle_nn_grad.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_double, _f64p]
    L.oracle_nn_grad.restype = ctypes.c_int
    return L


def _p(a, t):
    return a.ctypes.data_as(t)


def _series(T):
    return np.ascontiguousarray(T, dtype=np.float64)


def window_stats(T, m: int):
    """Per-window mean and population sigma, two passes (Eq. (4))."""
    T = _series(T)
    N = T.shape[0] - m + 1
    mu = np.empty(N)
    sd = np.empty(N)
    lib().oracle_window_stats(_p(T, _f64p), T.shape[0], m, _p(mu, _f64p), _p(sd, _f64p))
    return mu, sd


def drag(T, m: int, r: float, threads: int | None = None):
    """DRAG (Alg. 2) at one length: the range discords {i : P_m(i) >= r}.

    Returns (idx, nn, nnidx, evals) with idx in increasing order.
    ``threads`` selects the OpenMP build (same results, see merlin.c).
    """
    T = _series(T)
    N = T.shape[0] - m + 1
    idx = np.empty(N, dtype=np.int64)
    nn = np.empty(N)
    nnidx = np.empty(N, dtype=np.int64)
    cnt = ctypes.c_int64(0)
    ev = ctypes.c_uint64(0)
    rc = lib(threads).oracle_drag(_p(T, _f64p), T.shape[0], m, float(r), _p(idx, _i64p), _p(nn, _f64p),
                           _p(nnidx, _i64p), ctypes.byref(cnt), ctypes.byref(ev))
    if rc != 0:
        raise ValueError(f"oracle_drag failed rc={rc}")
    c = cnt.value
    return idx[:c].copy(), nn[:c].copy(), nnidx[:c].copy(), int(ev.value)


def nn_row(T, m: int, i: int):
    """Exact P_m(i) and its nearest non-self match j (smallest j on ties)."""
    T = _series(T)
    d = ctypes.c_double(0)
    j = ctypes.c_int64(0)
    rc = lib().oracle_nn_row(_p(T, _f64p), T.shape[0], m, int(i), ctypes.byref(d), ctypes.byref(j))
    if rc != 0:
        raise ValueError(f"oracle_nn_row failed rc={rc}")
    return float(d.value), int(j.value)


def merlin(T, minL: int, maxL: int, k: int, threads: int | None = None):
    """MERLIN (Alg. 1) driving DRAG; top-k discords per length.

    Returns a dict with idx, len, nn, nnidx (rows (m-minL)*k + rank), calls
    (DRAG invocations per length), r (successful r per length), evals.
    ``threads`` selects the OpenMP build (same results, see merlin.c).
    """
    T = _series(T)
    L = maxL - minL + 1
    idx = np.empty(L * k, dtype=np.int64)
    ln = np.empty(L * k, dtype=np.int32)
    nn = np.empty(L * k)
    nnidx = np.empty(L * k, dtype=np.int64)
    calls = np.empty(L, dtype=np.int32)
    rfin = np.empty(L)
    ev = ctypes.c_uint64(0)
    rc = lib(threads).oracle_merlin(_p(T, _f64p), T.shape[0], minL, maxL, k, _p(idx, _i64p),
                             _p(ln, _i32p), _p(nn, _f64p), _p(nnidx, _i64p), _p(calls, _i32p),
                             _p(rfin, _f64p), ctypes.byref(ev))
    if rc != 0:
        raise ValueError(f"oracle_merlin failed rc={rc}")
    return {"idx": idx, "len": ln, "nn": nn, "nnidx": nnidx, "calls": calls, "r": rfin,
            "evals": int(ev.value)}


def nn_grad(T, m: int, i: int, j: int, g: float = 1.0, out=None):
    """g * d P_m(i) / dT at a fixed neighbour j, accumulated into ``out``."""
    T = _series(T)
    if out is None:
        out = np.zeros(T.shape[0])
    rc = lib().oracle_nn_grad(_p(T, _f64p), T.shape[0], m, int(i), int(j), float(g), _p(out, _f64p))
    if rc != 0:
        raise ValueError(f"oracle_nn_grad failed rc={rc}")
    return out
