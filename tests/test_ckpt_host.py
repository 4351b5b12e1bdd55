"""Host-side pins of the checkpointed backtrace's window (no GPU): the cone
above a path cell holds the rest of the path within its block and every
predecessor of its cells, and the panel / chunk ranges the kernel computes
cover it. Also the bench's check for pairs too large for the oracle's sweep,
on small pairs: it accepts the oracle's own path and rejects a changed one."""
import numpy as np
import pytest

import bench
import oracle
from paper_2607_15478_amd import synth

STEPS = ((1, 1), (1, 2), (2, 1))


def cone(ie, je, r0):
    """Cells (r, c) of rows r0 .. ie with je - 2(ie - r) <= c <= je - ceil((ie - r)/2), c >= 0."""
    cells = set()
    for r in range(r0, ie + 1):
        a = ie - r
        for c in range(max(0, je - 2 * a), je - (a + 1) // 2 + 1):
            cells.add((r, c))
    return cells


@pytest.mark.parametrize("seed", range(6))
def test_cone_closed_under_predecessors(seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        r0 = int(rng.integers(0, 4)) * 16
        ie = r0 + int(rng.integers(0, 64))
        je = int(rng.integers(0, 300))
        C = cone(ie, je, r0)
        for (r, c) in C:
            for di, dj in STEPS:
                pr, pc = r - di, c - dj
                # inside the cone, or on the two checkpoint rows above the block,
                # or outside the matrix
                assert (pr, pc) in C or pr < r0 or pc < 0, ((ie, je, r0), (r, c), (pr, pc))


@pytest.mark.parametrize("n,m,K", [(1000, 1200, 16), (1000, 1200, 64), (1500, 1300, 256), (700, 860, 32)])
def test_path_cells_lie_in_their_block_cone(n, m, K):
    X, Y = synth.chroma_pair(n + m + K, n, m)
    _, path = oracle.align(X, Y)[:2]
    path = np.asarray(path)
    for r0, ie, je in bench.ckpt_block_entries(path, n, K):
        C = cone(ie, je, r0)
        inblock = path[(path[:, 0] >= r0) & (path[:, 0] <= ie)]
        for r, c in inblock:
            assert (int(r), int(c)) in C, (r0, ie, je, r, c)


@pytest.mark.parametrize("seed", range(6))
def test_kernel_ranges_cover_the_cone(seed):
    """The panels and 8-row chunks the window computes hold every cone cell;
    chunk ranges stay inside the block (k < 32 for K = 256)."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(15):
        K = int(rng.choice([16, 64, 256]))
        r0 = int(rng.integers(0, 4)) * K
        ie = r0 + int(rng.integers(0, K))
        je = int(rng.integers(0, 900))
        ranges = bench.ckpt_window_ranges(ie, je, r0)
        assert len(ranges) <= 2 * 256 // 64 + 2  # the kernel's wave count
        covered = set()
        for p, kbeg, kend in ranges:
            assert kbeg >= 0 and kend <= (ie - r0) // 8
            for k in range(kbeg, kend + 1):
                for r in range(r0 + 8 * k, r0 + 8 * k + 8):
                    for c in range(64 * p, 64 * p + 64):
                        covered.add((r, c))
        missing = [x for x in cone(ie, je, r0) if x not in covered]
        assert not missing, ((ie, je, r0), missing[:5])


def _large_check(monkeypatch, X, Y, path, total):
    monkeypatch.setattr(bench, "ORACLE_MAX_CELLS", 1e6)
    monkeypatch.setattr(bench, "ORACLE_SAMPLE_FRAMES", 500)
    _, val = bench.cpu_baseline_pair(X, Y, path, total)
    return val


def test_large_pair_check_accepts_the_oracle_path(monkeypatch):
    X, Y = synth.chroma_pair(21, 3000, 3600)
    total, path = oracle.align(X, Y)[:2]
    val = _large_check(monkeypatch, X, Y, np.asarray(path, dtype=np.int32), float(np.float32(total)))
    assert val["path_legal_rescored_and_segments_exact"], val["detail"]
    assert len(val["segments"]) == 5


def test_large_pair_check_rejects_a_changed_step(monkeypatch):
    """One (1,1),(1,2) pair of steps inside a sampled stretch swapped to
    (1,2),(1,1): still a legal path, no longer optimal. The stretch check
    must catch it even with the total taken from the changed path (so the
    rescoring alone cannot)."""
    X, Y = synth.chroma_pair(21, 3000, 3600)
    _, path = oracle.align(X, Y)[:2]
    path = np.asarray(path, dtype=np.int32).copy()
    d = np.diff(path, axis=0)
    k = next(k for k in range(200, 1400) if tuple(d[k]) == (1, 1) and tuple(d[k + 1]) == (1, 2))
    path[k + 1] = path[k] + np.array([1, 2])
    total = float(np.float32(oracle.path_cost(X, Y, path)))
    val = _large_check(monkeypatch, X, Y, path, total)
    assert not val["path_legal_rescored_and_segments_exact"]
    assert "mismatch" in val["detail"]


def test_large_pair_check_reports_the_totals_against_1e5(monkeypatch):
    """Both totals are judged against the FP64 re-score of the path at 1e-5,
    with no allowance growing with the path length: a total 2e-5 off fails,
    a compensated total equal to the re-score passes."""
    X, Y = synth.chroma_pair(21, 3000, 3600)
    total, path = oracle.align(X, Y)[:2]
    path = np.asarray(path, dtype=np.int32)
    monkeypatch.setattr(bench, "ORACLE_MAX_CELLS", 1e6)
    monkeypatch.setattr(bench, "ORACLE_SAMPLE_FRAMES", 500)
    _, val = bench.cpu_baseline_pair(X, Y, path, total * (1 + 2e-5), comp=total)
    assert val["path_legal_rescored_and_segments_exact"]
    assert val["total_within_1e-5"] is False and val["rel_bound"] == 1e-5
    assert val["compensated_total_within_1e-5"] is True
