"""Seeded synthetic inputs for the ParDTW workloads.

This module is shared by the CPU oracle tests and the GPU path. It only draws
numbers; it holds none of the alignment arithmetic (no cost, no dynamic
program, no backtrace, no gradient).

The paper evaluates on chroma features of piano recordings with a 23 ms hop and
cosine cost (Sec. IV) and times its implementations on random feature sequences
of length L (Sec. IV, Sec. VI-B/C). The recordings are not available, so the
generators below synthesise chroma-like sequences and a tempo-warped second
performance of the same material:

* ``chroma_like``: i.i.d. U[0,1] entries, a centred 5-frame moving average along
  time (edge frames replicated, length preserved), then each frame scaled to
  unit L2 norm.
* ``tempo_warp``: a piecewise-linear map tau from X-frame index to Y position
  with tau(0) = 0 and tau(N-1) = M-1. Breakpoints every U{50..200} X-frames;
  segment slopes U[lo, hi], then blended toward hi (or lo) by one scalar so the
  total span is exactly M-1 while every slope stays in [lo, hi]. Frame j of Y
  is X at position tau^-1(j), linearly interpolated between neighbouring
  frames.
* ``chroma_pair``: X chroma-like, Y = warp(X) + N(0, sigma) noise, clipped to
  [0, 1] and renormalised per frame.
* ``gaussian_pair``: X ~ N(0, 1), Y = warp(X) + N(0, sigma), no clip and no
  renormalisation (the differentiable/precision workload).

All randomness comes from numpy's PCG64 ``default_rng`` so the oracle and the
GPU path see bit-identical FP32 inputs.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "chroma_like",
    "tempo_warp_positions",
    "warp_copy",
    "chroma_pair",
    "gaussian_pair",
    "batch_lengths",
    "chroma_batch",
    "gaussian_batch",
    "WORKLOADS",
    "make_workload",
]


def chroma_like(rng: np.random.Generator, n: int, d: int = 12) -> np.ndarray:
    """Chroma-like frames: U[0,1], 5-frame centred moving average, unit L2 norm."""
    raw = rng.uniform(0.0, 1.0, size=(n, d))
    padded = np.concatenate([np.repeat(raw[:1], 2, 0), raw, np.repeat(raw[-1:], 2, 0)], 0)
    sm = (padded[0:n] + padded[1:n + 1] + padded[2:n + 2] + padded[3:n + 3] + padded[4:n + 4]) / 5.0
    nrm = np.linalg.norm(sm, axis=1, keepdims=True)
    return (sm / nrm).astype(np.float32)


def tempo_warp_positions(rng: np.random.Generator, n: int, m: int, lo: float, hi: float) -> np.ndarray:
    """Return, for each Y frame j in [0, m), its fractional X position tau^-1(j).

    tau is piecewise linear over X-frame index with breakpoints every U{50..200}
    frames and slopes in [lo, hi] adjusted by one scalar blend so that
    tau(n-1) = m-1 exactly. Requires lo <= (m-1)/(n-1) <= hi.
    """
    if n < 2 or m < 2:
        return np.zeros(m, dtype=np.float64)
    target = float(m - 1)
    span = float(n - 1)
    if not (lo * span - 1e-9 <= target <= hi * span + 1e-9):
        raise ValueError(f"slope range [{lo},{hi}] cannot map {n} frames onto {m}")
    # breakpoints along X
    bps = [0]
    while bps[-1] < n - 1:
        bps.append(min(n - 1, bps[-1] + int(rng.integers(50, 201))))
    xb = np.asarray(bps, dtype=np.float64)
    seg = np.diff(xb)
    s = rng.uniform(lo, hi, size=seg.shape[0])
    total = float(np.dot(s, seg))
    if total < target:
        room = float(np.dot(hi - s, seg))
        a = 0.0 if room <= 0 else (target - total) / room
        s = s + a * (hi - s)
    elif total > target:
        room = float(np.dot(s - lo, seg))
        a = 0.0 if room <= 0 else (total - target) / room
        s = s - a * (s - lo)
    yb = np.concatenate([[0.0], np.cumsum(s * seg)])
    yb[-1] = target  # remove accumulated rounding at the end point
    j = np.arange(m, dtype=np.float64)
    return np.interp(j, yb, xb)


def warp_copy(x: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """Linearly interpolate rows of x (float64 math) at fractional positions pos."""
    n = x.shape[0]
    x64 = x.astype(np.float64)
    p0 = np.clip(np.floor(pos).astype(np.int64), 0, n - 1)
    p1 = np.minimum(p0 + 1, n - 1)
    f = (pos - p0)[:, None]
    return x64[p0] * (1.0 - f) + x64[p1] * f


def chroma_pair(seed_or_rng, n: int, m: int, d: int = 12, lo: float = 0.8, hi: float = 1.25,
                sigma: float = 0.05):
    """(X, Y) chroma-like pair: Y is a tempo-warped noisy copy of X (FP32)."""
    rng = np.random.default_rng(seed_or_rng)
    x = chroma_like(rng, n, d)
    pos = tempo_warp_positions(rng, n, m, lo, hi)
    y = warp_copy(x, pos) + rng.normal(0.0, sigma, size=(m, d))
    y = np.clip(y, 0.0, 1.0)
    nrm = np.linalg.norm(y, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return x, (y / nrm).astype(np.float32)


def gaussian_pair(seed_or_rng, n: int, m: int, d: int = 128, lo: float = 0.8, hi: float = 1.25,
                  sigma: float = 0.05):
    """(X, Y) with X ~ N(0,1) and Y a tempo-warped copy plus N(0, sigma) noise."""
    rng = np.random.default_rng(seed_or_rng)
    x = rng.normal(0.0, 1.0, size=(n, d)).astype(np.float32)
    pos = tempo_warp_positions(rng, n, m, lo, hi)
    y = warp_copy(x, pos) + rng.normal(0.0, sigma, size=(m, d))
    return x, y.astype(np.float32)


def batch_lengths(rng: np.random.Generator, count: int, lo: int, hi: int, redraw_infeasible: bool):
    """Lengths (n_b, m_b) drawn uniformly in [lo, hi]; optionally redraw m until the
    pair admits a path under the (1,1),(1,2),(2,1) step set, i.e. m-1 <= 2(n-1)
    and n-1 <= 2(m-1)."""
    ns, ms = [], []
    for _ in range(count):
        n = int(rng.integers(lo, hi + 1))
        m = int(rng.integers(lo, hi + 1))
        while redraw_infeasible and (m - 1 > 2 * (n - 1) or n - 1 > 2 * (m - 1)):
            m = int(rng.integers(lo, hi + 1))
        ns.append(n)
        ms.append(m)
    return np.asarray(ns, dtype=np.int64), np.asarray(ms, dtype=np.int64)


def _warp_slopes(n: int, m: int):
    r = (m - 1) / max(n - 1, 1)
    return 0.8 * r, 1.25 * r


def chroma_batch(seed: int, count: int, lo: int, hi: int, d: int = 12, redraw_infeasible: bool = False):
    """Batch of chroma-like pairs with independent uniform lengths.

    Each pair gets its own generator from ``SeedSequence(seed).spawn``; the
    warp slopes are [0.8 r, 1.25 r] with r = (m-1)/(n-1)."""
    ss = np.random.SeedSequence(seed)
    master, *children = ss.spawn(count + 1)
    ns, ms = batch_lengths(np.random.default_rng(master), count, lo, hi, redraw_infeasible)
    pairs = []
    for b in range(count):
        lo_s, hi_s = _warp_slopes(int(ns[b]), int(ms[b]))
        pairs.append(chroma_pair(children[b], int(ns[b]), int(ms[b]), d, lo_s, hi_s))
    return pairs


def gaussian_batch(seed: int, count: int, lo: int, hi: int, d: int = 128):
    """Batch of Gaussian pairs; m is redrawn until the pair is feasible."""
    ss = np.random.SeedSequence(seed)
    master, *children = ss.spawn(count + 1)
    ns, ms = batch_lengths(np.random.default_rng(master), count, lo, hi, True)
    pairs = []
    for b in range(count):
        lo_s, hi_s = _warp_slopes(int(ns[b]), int(ms[b]))
        pairs.append(gaussian_pair(children[b], int(ns[b]), int(ms[b]), d, lo_s, hi_s))
    return pairs


# The five measured workloads. Sizes follow the paper's long-sequence regime
# (Sec. VI-C times 1k..100k frames; Sec. VI-D uses D = 12 chroma).
WORKLOADS = {
    "pair_1000x1200_d12": dict(kind="pair", seed=1, n=1000, m=1200, d=12, lo=0.8, hi=1.25),
    "pair_10000x12000_d12": dict(kind="pair", seed=2, n=10000, m=12000, d=12, lo=0.8, hi=1.25),
    "pair_50000x60000_d12": dict(kind="pair", seed=3, n=50000, m=60000, d=12, lo=0.7, hi=1.4),
    # past the code matrix's memory limit (3.6e11 cells: 360 GB of codes), for the checkpointed path
    "pair_600000x600000_d12": dict(kind="pair", seed=7, n=600000, m=600000, d=12, lo=0.8, hi=1.25),
    "pair_650000x650000_d12": dict(kind="pair", seed=8, n=650000, m=650000, d=12, lo=0.8, hi=1.25),
    "pair_1000000x1000000_d12": dict(kind="pair", seed=9, n=1000000, m=1000000, d=12, lo=0.8, hi=1.25),
    "pair_2800000x2800000_d12": dict(kind="pair", seed=10, n=2800000, m=2800000, d=12, lo=0.8, hi=1.25),
    "batch256_500to8000_d12": dict(kind="chroma_batch", seed=4, count=256, lo=500, hi=8000, d=12),
    # the same draw with infeasible pairs' m redrawn, so every pair is aligned
    "batch256_500to8000_d12_feasible": dict(kind="chroma_batch", seed=4, count=256, lo=500, hi=8000, d=12,
                                            redraw_infeasible=True),
    "batch32_2000to4000_d128": dict(kind="gaussian_batch", seed=5, count=32, lo=2000, hi=4000, d=128),
    # Segmental DTW of two 100k-frame sequences (Sec. VI-C times WSDTW on the GPU at 100k); the
    # number of fragments is a run parameter
    "segmental_100000x100000_d12": dict(kind="pair", seed=6, n=100000, m=100000, d=12, lo=0.8, hi=1.25),
    "segmental_50000x60000_d12": dict(kind="pair", seed=3, n=50000, m=60000, d=12, lo=0.7, hi=1.4),
}


def make_workload(name: str):
    """Materialise a named workload: a single (X, Y) pair or a list of pairs."""
    w = WORKLOADS[name]
    if w["kind"] == "pair":
        return chroma_pair(w["seed"], w["n"], w["m"], w["d"], w["lo"], w["hi"])
    if w["kind"] == "chroma_batch":
        return chroma_batch(w["seed"], w["count"], w["lo"], w["hi"], w["d"], w.get("redraw_infeasible", False))
    return gaussian_batch(w["seed"], w["count"], w["lo"], w["hi"], w["d"])
