"""Brute-force DTW by enumerating every legal warping path (tiny inputs only).

Written independently of the oracle: it never runs a dynamic program. A legal
path starts at (0,0), ends at (n-1,m-1) and takes steps (1,1), (1,2), (2,1);
its cost is C[0,0] plus, for every step, the step's weight (2, 3, 3) times the
cost of the cell it lands on (Sec. V of the paper; weight applied to the
destination cell, start cell weight 1).
"""
from __future__ import annotations

import numpy as np

STEPS = ((1, 1), (1, 2), (2, 1))  # codes 0, 1, 2
WEIGHTS = (2.0, 3.0, 3.0)


def enumerate_paths(n: int, m: int):
    """All legal paths as lists of step codes (forward order)."""
    out = []

    def rec(i, j, codes):
        if i == n - 1 and j == m - 1:
            out.append(list(codes))
            return
        for c, (di, dj) in enumerate(STEPS):
            if i + di <= n - 1 and j + dj <= m - 1:
                codes.append(c)
                rec(i + di, j + dj, codes)
                codes.pop()

    rec(0, 0, [])
    return out


def path_cells(codes):
    cells = [(0, 0)]
    for c in codes:
        di, dj = STEPS[c]
        cells.append((cells[-1][0] + di, cells[-1][1] + dj))
    return cells


def path_score(C: np.ndarray, codes) -> float:
    total = float(C[0, 0])
    i = j = 0
    for c in codes:
        di, dj = STEPS[c]
        i += di
        j += dj
        total += WEIGHTS[c] * float(C[i, j])
    return total


def brute_dtw(C: np.ndarray):
    """(J*, codes of the selected optimal path, number of optimal paths).

    Among all optimal paths, the selected one is the one whose step codes,
    read backward from the end, are lexicographically smallest: that is what
    a backtrace does when every cell keeps the lowest-index optimal step.
    Returns (inf, None, 0) when no legal path exists."""
    n, m = C.shape
    paths = enumerate_paths(n, m)
    if not paths:
        return float("inf"), None, 0
    scores = [path_score(C, p) for p in paths]
    best = min(scores)
    opt = [p for p, s in zip(paths, scores) if s == best]
    chosen = min(opt, key=lambda p: tuple(reversed(p)))
    return best, chosen, len(opt)
