"""Checkpointed DTW (the exact path without the code matrix; Sec. II-D names
memory as the limit on length and cites recomputation as the way past it):
the checkpoint rows against the FP64 oracle's D, and total, status and path
bit for bit those of the fused DP with the full code matrix, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2607_15478_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_15478_amd import pardtw as pd  # noqa: E402

DEV = "cuda:0"


def _features(seed, n, m, d):
    rng = np.random.default_rng(seed)
    X = synth.chroma_like(rng, n, d).astype(np.float32)
    Y = synth.chroma_like(rng, m, d).astype(np.float32)
    return X, Y


def _full(Xd, Yd):
    """The fused DP with the code matrix, then the backtrace."""
    n, m = Xd.shape[0], Yd.shape[0]
    w = pd.Workspace(n, m, DEV, cost=False)
    pd.align_into(Xd, Yd, w, fused=True)
    torch.cuda.synchronize()
    L = int(w.path_len.item())
    return float(w.total.item()), int(w.status.item()), w.path[:L].cpu().numpy()


def _ckpt(Xd, Yd, K, w=None):
    n, m = Xd.shape[0], Yd.shape[0]
    if w is None:
        w = pd.Workspace(n, m, DEV, cost=False, ckpt_rows=K)
    pd.align_into(Xd, Yd, w)
    torch.cuda.synchronize()
    L = int(w.path_len.item())
    return float(w.total.item()), int(w.status.item()), w.path[:L].cpu().numpy(), w


def _same(a, b):
    assert a[1] == b[1]
    assert a[0] == b[0] or (np.isinf(a[0]) and np.isinf(b[0]))
    assert np.array_equal(a[2], b[2])


SHAPES = [(1, 1), (2, 3), (7, 5), (16, 16), (17, 30), (31, 20), (32, 33), (33, 40), (63, 64), (64, 65), (65, 100),
          (130, 170), (255, 300), (256, 256), (257, 400), (333, 400), (600, 520), (777, 1500), (1000, 1200),
          (100, 199), (100, 250), (1500, 760)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("K", [16, 64, 256])
def test_ckpt_path_identical_to_full_codes(n, m, K):
    X, Y = _features(n * 13 + m + K, n, m, 12)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    _same(_ckpt(Xd, Yd, K)[:3], _full(Xd, Yd))


@pytest.mark.parametrize("d", [1, 5, 16])
@pytest.mark.parametrize("K", [32, 48, 240])
def test_ckpt_feature_widths_and_block_sizes(d, K):
    X, Y = _features(d * 7 + K, 900, 1100, d)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    _same(_ckpt(Xd, Yd, K)[:3], _full(Xd, Yd))


def test_ckpt_steep_pairs_and_zero_frames():
    """Slopes near 2 and 1/2 (paths along the band's edges) and zero frames (cost 1)."""
    for n, m in [(1000, 1998), (1998, 1000), (513, 1024), (1024, 513)]:
        X, Y = _features(n + 3 * m, n, m, 12)
        X[::97] = 0.0
        Y[5] = 0.0
        Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
        _same(_ckpt(Xd, Yd, 64)[:3], _full(Xd, Yd))


def test_ckpt_infeasible_pair():
    for n, m in [(10, 30), (30, 10), (2, 5)]:
        X, Y = _features(n + m, n, m, 12)
        Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
        tot, st, path, _ = _ckpt(Xd, Yd, 16)
        assert st == pd.PAIR_INFEASIBLE and np.isinf(tot) and len(path) == 0


def test_ckpt_workspace_reuse_across_sizes():
    """One workspace, a large pair then smaller ones: nothing a call leaves in
    the checkpoint buffer, the DP records or LDS changes the next result."""
    X, Y = _features(11, 3000, 3600, 12)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    w = pd.Workspace(3000, 3600, DEV, cost=False, ckpt_rows=128)
    _same(_ckpt(Xd, Yd, 128, w)[:3], _full(Xd, Yd))
    for n, m, seed in [(1000, 900, 12), (2999, 3001, 13)]:
        X2, Y2 = _features(seed, n, m, 12)
        X2d, Y2d = torch.from_numpy(X2).to(DEV), torch.from_numpy(Y2).to(DEV)
        pd.pardtw_dp_fused_ckpt(X2d, Y2d, 128, w.ckpt, w.total, w.status, w.ws)
        pd.pardtw_ckpt_backtrace(X2d, Y2d, 128, w.ckpt, w.status, w.path, w.path_len)
        torch.cuda.synchronize()
        L = int(w.path_len.item())
        _same((float(w.total.item()), int(w.status.item()), w.path[:L].cpu().numpy()), _full(X2d, Y2d))


@pytest.mark.parametrize("n,m,K", [(700, 800, 64), (1200, 1000, 256)])
def test_ckpt_rows_against_oracle_D(n, m, K):
    """Checkpoint rows bK-2, bK-1 on the band: the FP64 oracle's D within the
    totals' tolerance (FP32 sums of up to n terms)."""
    X, Y = _features(n + m + K, n, m, 12)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    _, _, _, w = _ckpt(Xd, Yd, K)
    ck = w.ckpt.cpu().numpy().reshape(-1, (-(-m // 64)) * 64)[:, :m]
    _, _, D = oracle.dtw_matrix(oracle.cost(X, Y), want_D=True)
    band = parity.band_mask(n, m)
    for b in range(1, (n - 1) // K + 1):
        for t, row in enumerate((b * K - 2, b * K - 1)):
            got = ck[2 * (b - 1) + t]
            sel = band[row]
            ref = D[row][sel]
            assert np.all(np.isfinite(ref))
            err = np.abs(got[sel].astype(np.float64) - ref)
            assert np.all(err <= parity.TOTAL_REL * np.abs(ref) + 1e-6), (row, float(err.max()))


@pytest.mark.parametrize("n,m", [(1000, 1200), (2000, 2400)])
def test_ckpt_against_oracle(n, m):
    X, Y = synth.chroma_pair(n + m, n, m)
    total, BP = oracle.dtw_features(X, Y)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    g_tot, g_st, g_path, _ = _ckpt(Xd, Yd, 256)
    assert g_st == pd.PAIR_OK
    parity.check_total(g_tot, total)
    parity.check_legal(g_path, n, m)
    parity.audit_path(g_path, BP, lambda c: oracle.probe(c, X=X, Y=Y)[0])


def test_ckpt_argument_errors():
    X, Y = _features(1, 100, 120, 12)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    w = pd.Workspace(100, 120, DEV, cost=False, ckpt_rows=16)
    for K in (0, 8, 17, 272):
        with pytest.raises(pd.PardtwError):
            pd.pardtw_dp_fused_ckpt(Xd, Yd, K, w.ckpt, w.total, w.status, w.ws)
        with pytest.raises(pd.PardtwError):
            pd.pardtw_ckpt_backtrace(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len)
    with pytest.raises(pd.PardtwError):  # checkpoint buffer too short
        pd.pardtw_dp_fused_ckpt(Xd, Yd, 16, w.ckpt[:-1], w.total, w.status, w.ws)
    Xw = torch.zeros((100, 17), dtype=torch.float32, device=DEV)
    Yw = torch.zeros((120, 17), dtype=torch.float32, device=DEV)
    with pytest.raises(pd.PardtwError):
        pd.pardtw_dp_fused_ckpt(Xw, Yw, 16, w.ckpt, w.total, w.status, w.ws)
    with pytest.raises(ValueError):
        pd.Workspace(100, 120, DEV, cost=False, ckpt_rows=20)


@pytest.mark.slow
def test_ckpt_full_size_identical():
    """50000 x 60000: the checkpointed path against the full code matrix."""
    X, Y = synth.make_workload("pair_50000x60000_d12")
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    ref = _full(Xd, Yd)
    got = _ckpt(Xd, Yd, 256)
    _same(got[:3], ref)


def test_ckpt_graph_capture_replays():
    """The checkpointed sweep and backtrace captured in a hipGraph: every
    replay, with eager work and clobbered outputs in between, gives the
    code-matrix path."""
    X, Y = _features(55, 1500, 1700, 12)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    ref = _full(Xd, Yd)
    w = pd.Workspace(1500, 1700, DEV, cost=False, ckpt_rows=128)
    _same(_ckpt(Xd, Yd, 128, w)[:3], ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pd.align_into(Xd, Yd, w)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pd.align_into(Xd, Yd, w)
    X2, Y2 = _features(56, 600, 700, 12)
    X2d, Y2d = torch.from_numpy(X2).to(DEV), torch.from_numpy(Y2).to(DEV)
    w2 = pd.Workspace(600, 700, DEV, cost=False, ckpt_rows=64)
    for rep in range(3):
        w.total.fill_(-1.0)
        w.status.fill_(-5)
        w.ckpt.fill_(7.0)
        w.path.fill_(-3)
        w.path_len.fill_(0)
        pd.align_into(X2d, Y2d, w2)
        g.replay()
        torch.cuda.synchronize()
        L = int(w.path_len.item())
        _same((float(w.total.item()), int(w.status.item()), w.path[:L].cpu().numpy()), ref)


@pytest.mark.parametrize("levels", [2, 3])
def test_ckpt_exact_ties(levels):
    """Features from a few repeated frames: many cells share one cost, and
    many candidate totals are exactly equal. The recomputed codes break every
    tie as the sweep does."""
    rng = np.random.default_rng(40 + levels)
    base = rng.integers(0, levels, size=(levels + 1, 12)).astype(np.float32) + 1.0
    X = base[rng.integers(0, levels + 1, size=900)]
    Y = base[rng.integers(0, levels + 1, size=1000)]
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    ref = _full(Xd, Yd)
    for K in (16, 128):
        _same(_ckpt(Xd, Yd, K)[:3], ref)


@pytest.mark.parametrize("n,m,K", [(5000, 6000, 16), (6000, 5000, 32), (20000, 24000, 256), (24000, 20000, 128)])
def test_ckpt_many_blocks(n, m, K):
    """Hundreds of blocks (and the walk across every block boundary) on
    tempo-warped pairs, against the code-matrix path."""
    X, Y = synth.chroma_pair(n + 2 * m + K, n, m)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    _same(_ckpt(Xd, Yd, K)[:3], _full(Xd, Yd))


def _ckpt_walks(Xd, Yd, K):
    """(one-workgroup checkpointed walk, split walk) over the same checkpoints."""
    n, m = Xd.shape[0], Yd.shape[0]
    w = pd.Workspace(n, m, DEV, cost=False, ckpt_rows=K)
    pd.pardtw_dp_fused_ckpt(Xd, Yd, K, w.ckpt, w.total, w.status, w.ws)
    out = []
    for par in (False, True):
        w.path.fill_(-9)
        w.path_len.fill_(-9)
        if par:
            ws = torch.full((pd.pardtw_ckpt_backtrace_parallel_bytes(n, m, K),), 0xEE, dtype=torch.uint8,
                            device=DEV)
            pd.pardtw_ckpt_backtrace_parallel(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len, ws)
        else:
            pd.pardtw_ckpt_backtrace(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len)
        torch.cuda.synchronize()
        L = int(w.path_len.item())
        out.append(w.path[:L].cpu().numpy())
    return out


@pytest.mark.parametrize("n,m,K,kind", [(3000, 3300, 32, "random"), (5000, 4000, 16, "random"),
                                        (9000, 10000, 64, "chroma"), (2100, 2000, 16, "chroma"),
                                        (1100, 1200, 64, "chroma")])
def test_ckpt_split_walk_equals_one_workgroup(n, m, K, kind):
    """The split walk over runs of blocks gives the one-workgroup walk's
    path: on chroma pairs (guessed starts pay) and on uniform random frames
    (optimal paths of nearby cells seldom merge, so runs are walked again)."""
    rng = np.random.default_rng(n + K)
    if kind == "random":
        X = rng.random((n, 12), dtype=np.float32)
        Y = rng.random((m, 12), dtype=np.float32)
    else:
        X, Y = synth.chroma_pair(n + m + K, n, m, 12, 0.8 * (m - 1) / (n - 1), 1.25 * (m - 1) / (n - 1))
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    ser, par = _ckpt_walks(Xd, Yd, K)
    assert len(ser) > 0 and np.array_equal(ser, par)
    # and the code-matrix path
    assert np.array_equal(par, _full(Xd, Yd)[2])


def test_ckpt_split_walk_workspace_check():
    X, Y = _features(61, 3000, 3100, 12)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    w = pd.Workspace(3000, 3100, DEV, cost=False, ckpt_rows=32)
    pd.pardtw_dp_fused_ckpt(Xd, Yd, 32, w.ckpt, w.total, w.status, w.ws)
    small = torch.empty(pd.pardtw_ckpt_backtrace_parallel_bytes(3000, 3100, 32) - 16, dtype=torch.uint8, device=DEV)
    with pytest.raises(pd.PardtwError, match="ERR_WORKSPACE"):
        pd.pardtw_ckpt_backtrace_parallel(Xd, Yd, 32, w.ckpt, w.status, w.path, w.path_len, small)
