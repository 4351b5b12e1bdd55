"""Seeded input generators: determinism and the stated recipe."""
import numpy as np
import pytest

from paper_2607_15478_amd import synth


def test_deterministic():
    a = synth.chroma_pair(1, 300, 360)
    b = synth.chroma_pair(1, 300, 360)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    assert a[0].dtype == np.float32 and a[1].dtype == np.float32


def test_chroma_frames_nonnegative_unit_norm():
    X, Y = synth.chroma_pair(2, 500, 600)
    for A in (X, Y):
        assert np.all(A >= 0)
        assert np.allclose(np.linalg.norm(A.astype(np.float64), axis=1), 1.0, atol=1e-6)


@pytest.mark.parametrize("n,m,lo,hi", [(1000, 1200, 0.8, 1.25), (5000, 6000, 0.7, 1.4), (800, 700, 0.8, 1.25)])
def test_warp_endpoints_and_slopes(n, m, lo, hi):
    rng = np.random.default_rng(3)
    pos = synth.tempo_warp_positions(rng, n, m, lo, hi)
    assert pos[0] == pytest.approx(0.0) and pos[-1] == pytest.approx(n - 1)
    dpos = np.diff(pos)  # X frames advanced per Y frame = 1 / slope
    assert np.all(dpos >= 1.0 / hi - 1e-9) and np.all(dpos <= 1.0 / lo + 1e-9)


def test_batch_lengths_and_feasibility_redraw():
    pairs = synth.gaussian_batch(5, 8, 2000, 4000, d=16)
    for X, Y in pairs:
        n, m = X.shape[0], Y.shape[0]
        assert 2000 <= n <= 4000 and 2000 <= m <= 4000
        assert m - 1 <= 2 * (n - 1) and n - 1 <= 2 * (m - 1)
    rng = np.random.default_rng(4)
    ns, ms = synth.batch_lengths(rng, 4000, 500, 8000, False)
    infeas = np.mean((ms - 1 > 2 * (ns - 1)) | (ns - 1 > 2 * (ms - 1)))
    # P(Y > 2X) + P(X > 2Y) for independent U[500, 8000] draws is about 0.436
    assert 0.40 < infeas < 0.47
