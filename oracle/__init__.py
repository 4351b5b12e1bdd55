"""FP64 CPU oracle for exact DTW / ParDTW -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and shares
no code with it; the two meet only through the seeded inputs of
``paper_2607_15478_amd.synth``.

The arithmetic lives in ``pardtw_oracle.c`` (plain loops, IEEE double, built
with gcc -O2 and no fast-math). This module is a ctypes wrapper around it plus
the closed-form feasibility test that follows from the step set.

It also holds subsequence DTW (weights 1, 1, 2 and a free start on the first
query row, Sec. II-B) and the segment-level step of Segmental DTW: NSDTW's
per-fragment minimum and WSDTW's ordered dynamic program over the stacked
fragment scores (Sec. II-C), plus the fragment split and the segment hop.

Parity status: every function here is pinned by ``tests/test_oracle.py`` and
``tests/test_oracle_segmental.py`` (brute-force path and placement
enumeration, closed forms, invariants, scipy's cosine distance, finite
differences, the exactness of the overlapping-chunk decomposition).
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
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC,
                               "-lm"])
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
        lib.oracle_dtw_features_mt.argtypes = [P, P, I, I, I, P, P, ctypes.c_int]
        lib.oracle_dtw_features_mt.restype = ctypes.c_int
        lib.oracle_probe.argtypes = [P, P, P, I, I, I, P, P, I, P, P]
        lib.oracle_probe.restype = ctypes.c_int
        lib.oracle_backtrace.argtypes = [P, I, I, P]
        lib.oracle_backtrace.restype = ctypes.c_int64
        lib.oracle_path_cost.argtypes = [P, P, I, I, I, P, I]
        lib.oracle_path_cost.restype = ctypes.c_double
        lib.oracle_path_grad.argtypes = [P, P, I, I, I, P, I, ctypes.c_double, P, P]
        lib.oracle_path_grad.restype = ctypes.c_int
        for name in ("oracle_subseq_matrix", "oracle_subseq_matrix_f32"):
            getattr(lib, name).argtypes = [P, I, I, P, P, P]
            getattr(lib, name).restype = ctypes.c_int
        lib.oracle_subseq_features.argtypes = [P, P, I, I, I, P, P]
        lib.oracle_subseq_features.restype = ctypes.c_int
        lib.oracle_subseq_probe.argtypes = [P, P, P, I, I, I, P, P, I, P, P]
        lib.oracle_subseq_probe.restype = ctypes.c_int
        lib.oracle_subseq_backtrace.argtypes = [P, I, I, I, P]
        lib.oracle_subseq_backtrace.restype = ctypes.c_int64
        lib.oracle_segment_ends.argtypes = [P, I, I, I, ctypes.c_int, P, P]
        lib.oracle_segment_ends.restype = ctypes.c_int
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


def dtw_features(X, Y, threads: int = 1):
    """DP with the cost computed row by row. Returns (total, BP int8 (n,m)).
    threads > 1 splits the columns of each row over that many OpenMP threads
    (bit-identical results)."""
    X, Y = _f32(X), _f32(Y)
    n, d = X.shape
    m = Y.shape[0]
    BP = np.empty((n, m), dtype=np.int8)
    tot = ctypes.c_double()
    lib = _load()
    if threads > 1:
        rc = lib.oracle_dtw_features_mt(_p(X), _p(Y), n, m, d, _p(BP), ctypes.byref(tot), int(threads))
    else:
        rc = lib.oracle_dtw_features(_p(X), _p(Y), n, m, d, _p(BP), ctypes.byref(tot))
    if rc != 0:
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


# --------------------------------------------------------------------------
# Subsequence DTW and Segmental DTW (Sec. II-B, II-C)
# --------------------------------------------------------------------------

SUB_WEIGHTS = {CODE_DIAG: 1.0, CODE_RIGHT: 1.0, CODE_DOWN: 2.0}
NSDTW, WSDTW = 0, 1


def subseq_reachable(i: int, j: int) -> bool:
    """Cell (i, j) lies on some subsequence path from the first query row:
    each step advances the reference by at least half the query advance, and
    the start column is free, so exactly when 2j >= i."""
    return 2 * j >= i


def subseq_matrix(C, want_D: bool = False):
    """Subsequence DP over a given cost matrix (FP64, or FP32 widened exactly).
    Returns (S float64 (m,), BP int8 (n,m), D float64 (n,m) or None)."""
    C = np.asarray(C)
    n, m = C.shape
    BP = np.empty((n, m), dtype=np.int8)
    S = np.empty(m, dtype=np.float64)
    D = np.empty((n, m), dtype=np.float64) if want_D else None
    lib = _load()
    if C.dtype == np.float32:
        C = np.ascontiguousarray(C)
        rc = lib.oracle_subseq_matrix_f32(_p(C), n, m, _p(D) if want_D else None, _p(BP), _p(S))
    else:
        C = np.ascontiguousarray(C, dtype=np.float64)
        rc = lib.oracle_subseq_matrix(_p(C), n, m, _p(D) if want_D else None, _p(BP), _p(S))
    if rc != 0:
        raise MemoryError("oracle_subseq_matrix")
    return S, BP, D


def subseq_features(X, Y):
    """Subsequence DP with the cost computed row by row: (S (m,), BP (n,m))."""
    X, Y = _f32(X), _f32(Y)
    n, d = X.shape
    m = Y.shape[0]
    BP = np.empty((n, m), dtype=np.int8)
    S = np.empty(m, dtype=np.float64)
    if _load().oracle_subseq_features(_p(X), _p(Y), n, m, d, _p(BP), _p(S)) != 0:
        raise MemoryError("oracle_subseq_features")
    return S, BP


def subseq_probe(cells, X=None, Y=None, C32=None):
    """FP64 candidate totals (k, 3) and D (k,) of the subsequence DP at the
    given cells, from features or from an FP32 cost matrix."""
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
        rc = lib.oracle_subseq_probe(None, None, _p(C32), n, m, 0, _p(ci), _p(cj), k, _p(cand), _p(dval))
    else:
        X, Y = _f32(X), _f32(Y)
        n, d = X.shape
        m = Y.shape[0]
        rc = lib.oracle_subseq_probe(_p(X), _p(Y), None, n, m, d, _p(ci), _p(cj), k, _p(cand), _p(dval))
    if rc != 0:
        raise RuntimeError(f"oracle_subseq_probe failed ({rc})")
    out_c = np.empty_like(cand)
    out_d = np.empty_like(dval)
    out_c[order] = cand
    out_d[order] = dval
    return out_c, out_d


def subseq_backtrace(BP, end: int) -> np.ndarray:
    """Forward subsequence path (L, 2) from the first query row to
    (n-1, end); empty when that cell is unreachable."""
    BP = np.ascontiguousarray(BP, dtype=np.int8)
    n, m = BP.shape
    path = np.empty((n, 2), dtype=np.int32)
    L = _load().oracle_subseq_backtrace(_p(BP), n, m, int(end), _p(path))
    if L < 0:
        raise RuntimeError("oracle_subseq_backtrace: malformed backtrace matrix")
    return path[:L].copy()


def subseq_path_score(C, path) -> float:
    """FP64 score of a subsequence path over a cost matrix: C at the start
    cell plus, per step, the step's weight (1, 1, 2) times the cost it lands
    on. NaN when the path is not a legal subsequence path."""
    C = np.asarray(C, dtype=np.float64)
    path = np.asarray(path).reshape(-1, 2)
    if len(path) == 0 or path[0][0] != 0:
        return float("nan")
    total = float(C[path[0][0], path[0][1]])
    steps = {(1, 1): 1.0, (1, 2): 1.0, (2, 1): 2.0}
    for a, b in zip(path[:-1], path[1:]):
        w = steps.get((int(b[0] - a[0]), int(b[1] - a[1])))
        if w is None:
            return float("nan")
        total += w * float(C[b[0], b[1]])
    return total


def fragment_starts(la: int, nfrag: int) -> np.ndarray:
    """Row where each of the nfrag fragments of a length-la sequence starts,
    plus la at the end: fragment f is rows [floor(f la / N), floor((f+1) la / N)),
    lengths differing by at most one (Sec. II-B: approximately equal)."""
    if nfrag < 1 or la < nfrag:
        raise ValueError("need 1 <= nfrag <= la")
    return np.array([(f * la) // nfrag for f in range(nfrag + 1)], dtype=np.int64)


def segment_hop(la: int, nfrag: int) -> int:
    """Column advance of a segment-level match: the shortest stretch of the
    reference a fragment of la / N frames can match under a warping factor of
    at most 2 (Sec. II-C), la / (2N) rounded down, and at least one column so
    that the fragment ends stay strictly increasing."""
    return max(1, la // (2 * nfrag))


def segment_ends(S, hop: int, variant: int):
    """Fragment end columns from the stacked scores S (nf, m):
    returns (total, ends int64 (nf,)); see oracle_segment_ends."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    nf, m = S.shape
    ends = np.empty(nf, dtype=np.int64)
    tot = ctypes.c_double()
    if _load().oracle_segment_ends(_p(S), nf, m, int(hop), int(variant), _p(ends), ctypes.byref(tot)) != 0:
        raise RuntimeError("oracle_segment_ends failed")
    return tot.value, ends


def subseq_chunked(C, nchunks: int) -> np.ndarray:
    """Scores S of a subsequence DP computed as the paper's overlapping
    reference chunks (Sec. III-A, second dimension): chunk c owns end columns
    [a_c, b_c) and sweeps only reference columns [a_c - 2(n-1), b_c), the
    widest stretch a path ending in the chunk can cover. The result must equal
    the whole-reference sweep exactly."""
    C = np.asarray(C, dtype=np.float64)
    n, m = C.shape
    S = np.empty(m, dtype=np.float64)
    bounds = [(c * m) // nchunks for c in range(nchunks + 1)]
    for c in range(nchunks):
        a, b = bounds[c], bounds[c + 1]
        if a == b:
            continue
        lo = max(0, a - 2 * (n - 1))
        s_loc, _, _ = subseq_matrix(C[:, lo:b])
        S[a:b] = s_loc[a - lo:]
    return S


def segmental(X, Y, nfrag: int, variant: int = WSDTW):
    """Segmental DTW of feature sequences X (A, la x d) and Y (B, lb x d).
    Returns a dict with the total, the fragment ends, each fragment's path in
    global coordinates, their concatenation, the stacked scores S and the
    per-fragment backtrace matrices (Sec. II-B/II-C, steps 1-5)."""
    X, Y = _f32(X), _f32(Y)
    la = X.shape[0]
    starts = fragment_starts(la, nfrag)
    rows, bps = [], []
    for f in range(nfrag):
        s_f, bp_f = subseq_features(X[starts[f]:starts[f + 1]], Y)
        rows.append(s_f)
        bps.append(bp_f)
    S = np.stack(rows)
    hop = segment_hop(la, nfrag)
    total, ends = segment_ends(S, hop, variant)
    paths = []
    for f in range(nfrag):
        if ends[f] < 0:
            paths.append(np.empty((0, 2), np.int32))
            continue
        p = subseq_backtrace(bps[f], ends[f]).astype(np.int64)
        p[:, 0] += starts[f]
        paths.append(p.astype(np.int32))
    path = np.concatenate(paths) if paths else np.empty((0, 2), np.int32)
    return {"total": total, "ends": ends, "paths": paths, "path": path, "S": S, "BP": bps,
            "starts": starts, "hop": hop}
