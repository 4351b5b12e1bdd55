"""Path and backtrace parity checks between the GPU results and the oracle.

Rules (restating the parity contract of the build):

* a GPU path must be legal: start (0,0), end (N-1,M-1), every step in
  {(1,1), (1,2), (2,1)};
* walking the GPU path backward, the step taken into each cell must equal the
  oracle's backtrace code at that cell, unless the two candidate totals are a
  declared near-tie: |cand_r - cand_r'| < 1e-6 * max(|cand_r|, |cand_r'|, 1),
  evaluated on the oracle's FP64 candidates;
* the FP32 total must be within 1e-5 relative of the oracle's FP64 total;
* the GPU path re-scored in FP64 must not exceed J* (1 + 1e-6) + 1e-9.
"""
from __future__ import annotations

import numpy as np

STEPS = ((1, 1), (1, 2), (2, 1))
TIE_REL = 1e-6
TOTAL_REL = 1e-5


def step_codes(path: np.ndarray) -> np.ndarray:
    d = np.diff(path.astype(np.int64), axis=0)
    codes = np.full(len(d), -1, dtype=np.int64)
    for c, (di, dj) in enumerate(STEPS):
        codes[(d[:, 0] == di) & (d[:, 1] == dj)] = c
    return codes


def check_legal(path: np.ndarray, n: int, m: int):
    assert path.ndim == 2 and path.shape[1] == 2 and len(path) >= 1
    assert tuple(path[0]) == (0, 0), "path must start at (0,0)"
    assert tuple(path[-1]) == (n - 1, m - 1), "path must end at (N-1,M-1)"
    codes = step_codes(path)
    assert np.all(codes >= 0), "illegal step in path"
    assert len(path) <= min(n, m)


def is_tie(cand: np.ndarray, r: int, r2: int) -> bool:
    a, b = float(cand[r]), float(cand[r2])
    if not (np.isfinite(a) and np.isfinite(b)):
        return False
    return abs(a - b) < TIE_REL * max(abs(a), abs(b), 1.0)


def audit_path(path: np.ndarray, oracle_bp: np.ndarray, cand_at):
    """Compare the GPU path's steps with the oracle's codes.

    cand_at(cells (k,2)) -> (k,3) FP64 candidate totals. Returns the number of
    declared near-ties; raises AssertionError on a real mismatch."""
    codes = step_codes(path)
    cells = path[1:]
    ocodes = oracle_bp[cells[:, 0], cells[:, 1]].astype(np.int64)
    diff = np.nonzero(ocodes != codes)[0]
    if len(diff) == 0:
        return 0
    cands = cand_at(cells[diff])
    for q, k in enumerate(diff):
        r_gpu, r_or = int(codes[k]), int(ocodes[k])
        assert 0 <= r_or <= 2, f"GPU path enters cell {tuple(cells[k])} that the oracle marks unreachable"
        assert is_tie(cands[q], r_or, r_gpu), (
            f"step mismatch at {tuple(cells[k])}: gpu {r_gpu} oracle {r_or}, candidates {cands[q]}")
    return len(diff)


def audit_bp_matrix(gpu_bp: np.ndarray, oracle_bp: np.ndarray, D: np.ndarray, C: np.ndarray):
    """Full backtrace-matrix parity: every differing cell must be a declared tie
    of the oracle's FP64 candidates (computed from the full D). Returns the
    number of tie cells."""
    diff = np.argwhere(gpu_bp != oracle_bp)
    for i, j in diff:
        cand = np.full(3, np.inf)
        for r, (di, dj) in enumerate(STEPS):
            if i - di >= 0 and j - dj >= 0:
                cand[r] = D[i - di, j - dj] + (2.0 if r == 0 else 3.0) * float(C[i, j])
        assert 0 <= gpu_bp[i, j] <= 2 and 0 <= oracle_bp[i, j] <= 2, (
            f"code mismatch at {(i, j)} involving an unreachable cell: gpu {gpu_bp[i, j]} oracle {oracle_bp[i, j]}")
        assert is_tie(cand, int(oracle_bp[i, j]), int(gpu_bp[i, j])), (
            f"code mismatch at {(i, j)}: gpu {gpu_bp[i, j]} oracle {oracle_bp[i, j]} candidates {cand}")
    return len(diff)


def band_mask(n: int, m: int) -> np.ndarray:
    """(n, m) bool: cells that can lie on a path from (0,0) to (n-1,m-1) with
    the steps (1,1), (1,2), (2,1): reachable from the origin (j <= 2i and
    i <= 2j) and able to reach the end ((m-1-j) <= 2(n-1-i) and
    (n-1-i) <= 2(m-1-j)). The DP defines codes on these cells only."""
    i = np.arange(n)[:, None]
    j = np.arange(m)[None, :]
    fwd = (j <= 2 * i) & (i <= 2 * j)
    ri, rj = n - 1 - i, m - 1 - j
    end = (rj <= 2 * ri) & (ri <= 2 * rj)
    return fwd & end


def band_groups(n: int, m: int) -> np.ndarray:
    """(P, G) bool: 8-row group k of 64-column panel p holds a real cell
    reachable from the origin and a real cell from which (n-1,m-1) is
    reachable (enumerated cell by cell): the groups the band layout writes."""
    P, G = -(-m // 64), -(-n // 8)
    i = np.arange(n)[:, None]
    j = np.arange(m)[None, :]
    fwd = (j <= 2 * i) & (i <= 2 * j)
    ri, rj = n - 1 - i, m - 1 - j
    end = (rj <= 2 * ri) & (ri <= 2 * rj)
    def per_group(mask):
        pad = np.zeros((G * 8, P * 64), dtype=bool)
        pad[:n, :m] = mask
        return pad.reshape(G, 8, P, 64).any(axis=(1, 3)).T
    return per_group(fwd) & per_group(end)


def subseq_band_mask(n: int, m: int) -> np.ndarray:
    """(n, m) bool: cells that can lie on a subsequence path (Sec. II-B), which
    starts anywhere on row 0 and ends anywhere on row n-1: row 0 reaches the
    cell (i <= 2j) and the cell reaches row n-1 inside the matrix
    ((n-1-i) <= 2(m-1-j)). The subsequence DP defines codes on these cells."""
    i = np.arange(n)[:, None]
    j = np.arange(m)[None, :]
    return (i <= 2 * j) & ((n - 1 - i) <= 2 * (m - 1 - j))


def subseq_band_groups(n: int, m: int) -> np.ndarray:
    """(P, G) bool: group k of panel p holds a real cell that row 0 reaches and
    a real cell that reaches row n-1 (enumerated cell by cell)."""
    P, G = -(-m // 64), -(-n // 8)
    i = np.arange(n)[:, None]
    j = np.arange(m)[None, :]
    def per_group(mask):
        pad = np.zeros((G * 8, P * 64), dtype=bool)
        pad[:n, :m] = mask
        return pad.reshape(G, 8, P, 64).any(axis=(1, 3)).T
    return per_group(i <= 2 * j) & per_group((n - 1 - i) <= 2 * (m - 1 - j))


def check_total(gpu_total: float, oracle_total: float):
    if not np.isfinite(oracle_total):
        assert not np.isfinite(gpu_total)
        return
    assert abs(gpu_total - oracle_total) <= TOTAL_REL * abs(oracle_total) + 1e-6, (gpu_total, oracle_total)


def to_panel(C: np.ndarray) -> np.ndarray:
    """Row-major (n, m) cost to the panel layout (flat): 64-column panels,
    8-row groups; a group holds rows 0-3 of its 64 columns, then rows 4-7,
    with each column's 4 rows contiguous."""
    n, m = C.shape
    P, G = -(-m // 64), -(-n // 8)
    pad = np.zeros((G * 8, P * 64), dtype=C.dtype)
    pad[:n, :m] = C
    # [G, 2, 4, P, 64] -> [P, G, 2, 64, 4]
    return pad.reshape(G, 2, 4, P, 64).transpose(3, 0, 1, 4, 2).reshape(-1).copy()


def from_panel(flat: np.ndarray, n: int, m: int) -> np.ndarray:
    P, G = -(-m // 64), -(-n // 8)
    a = flat[: P * G * 512].reshape(P, G, 2, 64, 4)
    return a.transpose(1, 2, 4, 0, 3).reshape(G * 8, P * 64)[:n, :m]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def to_bp_layout(B: np.ndarray) -> np.ndarray:
    """Row-major (n, m) int8 codes to the DP's backtrace layout (flat uint8):
    64-column panels, 8-row groups, a column's 8 codes contiguous."""
    n, m = B.shape
    P, G = -(-m // 64), -(-n // 8)
    pad = np.full((G * 8, P * 64), 3, dtype=np.uint8)
    pad[:n, :m] = B
    # [G, 8, P, 64] -> [P, G, 64, 8]
    return pad.reshape(G, 8, P, 64).transpose(2, 0, 3, 1).reshape(-1).copy()


def random_path(n: int, m: int, rng: np.random.Generator, mean_run: float = 50.0) -> np.ndarray:
    """A random legal path from (0,0) to (n-1,m-1) made of runs of one
    preferred step (so it also holds long stretches at slope 1/2 and 2)."""
    steps = ((1, 1), (1, 2), (2, 1))

    def ok(ri, rj):
        return (ri == 0 and rj == 0) or (ri >= 1 and rj >= 1 and rj <= 2 * ri and ri <= 2 * rj)

    i = j = 0
    out = [(0, 0)]
    pref, run = 0, 0
    while (i, j) != (n - 1, m - 1):
        if run <= 0:
            pref, run = int(rng.integers(0, 3)), int(rng.geometric(1.0 / mean_run))
        run -= 1
        order = [pref] + [int(s) for s in rng.permutation(3) if s != pref]
        for s in order:
            di, dj = steps[s]
            if ok(n - 1 - i - di, m - 1 - j - dj):
                i, j = i + di, j + dj
                break
        else:  # pragma: no cover - a feasible remainder always admits a step
            raise AssertionError("no legal step")
        out.append((i, j))
    return np.array(out, dtype=np.int32)


def bp_with_path(n: int, m: int, path: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Random codes everywhere, the path's own step codes on its cells, 3 at
    the origin."""
    B = rng.integers(0, 4, size=(n, m), dtype=np.uint8)
    codes = step_codes(path)
    B[path[1:, 0], path[1:, 1]] = codes.astype(np.uint8)
    B[0, 0] = 3
    return B


def path_deviation(path_a: np.ndarray, path_b: np.ndarray, n: int):
    """Mean and max over X-frames i of |j_A(i) - j_B(i)|, each path's j taken
    at its cell in row i, linearly interpolated over rows the path skips."""
    rows = np.arange(n, dtype=np.float64)
    ja = np.interp(rows, path_a[:, 0].astype(np.float64), path_a[:, 1].astype(np.float64))
    jb = np.interp(rows, path_b[:, 0].astype(np.float64), path_b[:, 1].astype(np.float64))
    dev = np.abs(ja - jb)
    return float(dev.mean()), float(dev.max())
