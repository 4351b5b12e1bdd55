"""FP64 CPU oracle for exact DTW / ParDTW -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and shares
no code with it; the two meet only through the seeded inputs of
``paper_2607_15478_amd.synth``.

The arithmetic lives in ``pardtw_oracle.c`` (plain loops, IEEE double, built
with gcc -O2 and no fast-math). This module is a ctypes wrapper around it plus
the closed-form feasibility test that follows from the step set.

Parity status: every function here is pinned by ``tests/test_oracle.py``
(brute-force path enumeration, closed forms, invariants, scipy's cosine
distance, finite differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pardtw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CODE_DIAG, CODE_RIGHT, CODE_DOWN, CODE_NONE = 0, 1, 2, 3
STEPS = {CODE_DIAG: (1, 1), CODE_RIGHT: (1, 2), CODE_DOWN: (2, 1)}
WEIGHTS = {CODE_DIAG: 2.0, CODE_RIGHT: 3.0, CODE_DOWN: 3.0}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.oracle_cost.argtypes = [P, P, I, I, I, P]
        lib.oracle_cost.restype = ctypes.c_int
        lib.oracle_dtw_matrix.argtypes = [P, I, I, P, P, P]
        lib.oracle_dtw_matrix.restype = ctypes.c_int
        lib.oracle_dtw_matrix_f32.argtypes = [P, I, I, P, P, P]
        lib.oracle_dtw_matrix_f32.restype = ctypes.c_int
        lib.oracle_dtw_features.argtypes = [P, P, I, I, I, P, P]
        lib.oracle_dtw_features.restype = ctypes.c_int
        lib.oracle_probe.argtypes = [P, P, P, I, I, I, P, P, I, P, P]
        lib.oracle_probe.restype = ctypes.c_int
        lib.oracle_backtrace.argtypes = [P, I, I, P]
        lib.oracle_backtrace.restype = ctypes.c_int64
        lib.oracle_path_cost.argtypes = [P, P, I, I, I, P, I]
        lib.oracle_path_cost.restype = ctypes.c_double
        lib.oracle_path_grad.argtypes = [P, P, I, I, I, P, I, ctypes.c_double, P, P]
        lib.oracle_path_grad.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def feasible(n: int, m: int) -> bool:
    """A legal path from (0,0) to (n-1,m-1) exists iff the end is reachable:
    each step advances one coordinate by 1 and the other by 1 or 2, so
    m-1 <= 2(n-1) and n-1 <= 2(m-1) (and n, m >= 1)."""
    return n >= 1 and m >= 1 and (m - 1) <= 2 * (n - 1) and (n - 1) <= 2 * (m - 1)


def cost(X, Y) -> np.ndarray:
    """FP64 cosine-distance matrix (n, m) from FP32 features."""
    X, Y = _f32(X), _f32(Y)
    n, d = X.shape
    m = Y.shape[0]
    C = np.empty((n, m), dtype=np.float64)
    if _load().oracle_cost(_p(X), _p(Y), n, m, d, _p(C)) != 0:
        raise MemoryError("oracle_cost")
    return C


def dtw_matrix(C, want_D: bool = False):
    """DP over a given cost matrix. FP64 input runs as is; FP32 input is
    widened exactly. Returns (total, BP int8 (n,m), D float64 (n,m) or None)."""
    C = np.asarray(C)
    n, m = C.shape
    BP = np.empty((n, m), dtype=np.int8)
    D = np.empty((n, m), dtype=np.float64) if want_D else None
    tot = ctypes.c_double()
    lib = _load()
    if C.dtype == np.float32:
        C = np.ascontiguousarray(C)
        rc = lib.oracle_dtw_matrix_f32(_p(C), n, m, _p(D) if want_D else None, _p(BP), ctypes.byref(tot))
    else:
        C = np.ascontiguousarray(C, dtype=np.float64)
        rc = lib.oracle_dtw_matrix(_p(C), n, m, _p(D) if want_D else None, _p(BP), ctypes.byref(tot))
    if rc != 0:
        raise MemoryError("oracle_dtw_matrix")
    return tot.value, BP, D


def dtw_features(X, Y):
    """DP with the cost computed row by row. Returns (total, BP int8 (n,m))."""
    X, Y = _f32(X), _f32(Y)
    n, d = X.shape
    m = Y.shape[0]
    BP = np.empty((n, m), dtype=np.int8)
    tot = ctypes.c_double()
    if _load().oracle_dtw_features(_p(X), _p(Y), n, m, d, _p(BP), ctypes.byref(tot)) != 0:
        raise MemoryError("oracle_dtw_features")
    return tot.value, BP


def backtrace(BP) -> np.ndarray:
    """Forward path (L, 2) int32 from (0,0) to (n-1,m-1); empty when the end
    cell is unreachable."""
    BP = np.ascontiguousarray(BP, dtype=np.int8)
    n, m = BP.shape
    path = np.empty((min(n, m), 2), dtype=np.int32)
    L = _load().oracle_backtrace(_p(BP), n, m, _p(path))
    if L < 0:
        raise RuntimeError("oracle_backtrace: malformed backtrace matrix")
    return path[:L].copy()


def align(X, Y):
    """Exact DTW of two feature sequences: (total, path, BP)."""
    total, BP = dtw_features(X, Y)
    path = backtrace(BP) if np.isfinite(total) else np.empty((0, 2), np.int32)
    return total, path, BP


def probe(cells, X=None, Y=None, C32=None):
    """FP64 candidate totals (k, 3) and accumulated costs (k,) at the given
    cells (k, 2), from a fresh sweep over features or over an FP32 cost."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 2)
    order = np.argsort(cells[:, 0], kind="stable")
    ci = np.ascontiguousarray(cells[order, 0])
    cj = np.ascontiguousarray(cells[order, 1])
    k = len(ci)
    cand = np.empty((k, 3), dtype=np.float64)
    dval = np.empty(k, dtype=np.float64)
    lib = _load()
    if C32 is not None:
        C32 = _f32(C32)
        n, m = C32.shape
        rc = lib.oracle_probe(None, None, _p(C32), n, m, 0, _p(ci), _p(cj), k, _p(cand), _p(dval))
    else:
        X, Y = _f32(X), _f32(Y)
        n, d = X.shape
        m = Y.shape[0]
        rc = lib.oracle_probe(_p(X), _p(Y), None, n, m, d, _p(ci), _p(cj), k, _p(cand), _p(dval))
    if rc != 0:
        raise RuntimeError(f"oracle_probe failed ({rc})")
    out_c = np.empty_like(cand)
    out_d = np.empty_like(dval)
    out_c[order] = cand
    out_d[order] = dval
    return out_c, out_d


def path_cost(X, Y, path) -> float:
    """FP64 cost of a path (NaN if it is not a legal full path)."""
    X, Y = _f32(X), _f32(Y)
    path = np.ascontiguousarray(path, dtype=np.int32).reshape(-1, 2)
    n, d = X.shape
    m = Y.shape[0]
    return _load().oracle_path_cost(_p(X), _p(Y), n, m, d, _p(path), len(path))


def path_grad(X, Y, path, g: float = 1.0):
    """FP64 gradient (dX, dY) of g * J(path) with the path held fixed."""
    X, Y = _f32(X), _f32(Y)
    path = np.ascontiguousarray(path, dtype=np.int32).reshape(-1, 2)
    n, d = X.shape
    m = Y.shape[0]
    dX = np.empty((n, d), dtype=np.float64)
    dY = np.empty((m, d), dtype=np.float64)
    _load().oracle_path_grad(_p(X), _p(Y), n, m, d, _p(path), len(path), float(g), _p(dX), _p(dY))
    return dX, dY
