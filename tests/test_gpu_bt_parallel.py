"""The split backtrace (pardtw_backtrace_parallel and its packed-code form)
against the serial walk: the same path, cell for cell, and the same length,
on chroma pairs (paths merge fast: the guesses pay), on random costs and on
hand-made code matrices (paths wander: the final check walks segments
again), and on corrupt codes (both walks fail)."""
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


def _paths(bp, n, m, status, packed=False):
    """(serial path, split path) over the same codes."""
    out = []
    for par in (False, True):
        path = torch.full((min(n, m), 2), -7, dtype=torch.int32, device=DEV)
        plen = torch.full((1,), -7, dtype=torch.int32, device=DEV)
        if par:
            ws = torch.full((pd.pardtw_backtrace_parallel_bytes(n, m),), 0xEE, dtype=torch.uint8, device=DEV)
            pd.pardtw_backtrace_parallel(bp, n, m, status, path, plen, ws, packed=packed)
        elif packed:
            pd.pardtw_backtrace_packed(bp, n, m, status, path, plen)
        else:
            pd.pardtw_backtrace(bp, n, m, status, path, plen)
        torch.cuda.synchronize()
        L = int(plen.item())
        out.append(path[:L].cpu().numpy())
    return out


def _dp_codes(C, packed=False):
    n, m = C.shape
    Cd = torch.from_numpy(parity.to_panel(C)).to(DEV)
    nb = pd.pardtw_bp2_bytes(n, m) if packed else pd.pardtw_bp_bytes(n, m)
    bp = torch.empty(nb, dtype=torch.uint8, device=DEV)
    ws = torch.zeros(pd.pardtw_dp_workspace_bytes(n, m), dtype=torch.uint8, device=DEV)
    total = torch.empty(1, dtype=torch.float32, device=DEV)
    st = torch.empty(1, dtype=torch.int32, device=DEV)
    (pd.pardtw_dp_packed if packed else pd.pardtw_dp)(Cd, n, m, bp, total, st, ws, pd.LAYOUT_PANEL)
    return bp, st


SHAPES = [(1, 1), (2, 3), (9, 17), (100, 199), (511, 600), (512, 700), (513, 513), (1000, 1200), (1023, 1800),
          (1025, 900), (3000, 2600), (5000, 9000), (12000, 10000)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("packed", [False, True])
def test_split_walk_equals_serial_on_chroma(n, m, packed):
    rng = np.random.default_rng(3 * n + m)
    X, Y = synth.chroma_like(rng, n), synth.chroma_like(rng, m)
    w = pd.Workspace(n, m, DEV, packed=packed)
    pd.align_into(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), w, fused=True, serial_backtrace=True)
    ser, par = _paths(w.bp, n, m, w.status, packed)
    assert len(ser) > 0 or (n, m) in ((1, 1),) or not parity.band_mask(n, m).any()
    assert np.array_equal(ser, par)


@pytest.mark.parametrize("n,m,seed", [(2000, 2500, 1), (4000, 3000, 2), (7000, 9000, 3)])
@pytest.mark.parametrize("packed", [False, True])
def test_split_walk_equals_serial_on_random_costs(n, m, seed, packed):
    """Uniform random costs: optimal paths of nearby cells merge slowly, so
    guesses miss and segments are walked again."""
    C = np.random.default_rng(seed).random((n, m), dtype=np.float32)
    bp, st = _dp_codes(C, packed)
    ser, par = _paths(bp, n, m, st, packed)
    assert len(ser) > 0
    assert np.array_equal(ser, par)


def _pack_bytes(codes: np.ndarray) -> np.ndarray:
    """Row-major int8 codes to the DP's byte layout (64-column panels, 8-row groups)."""
    n, m = codes.shape
    P, G = -(-m // 64), -(-n // 8)
    bp = np.zeros(P * G * 512, dtype=np.uint8)
    i, j = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
    idx = (((j // 64) * G + i // 8) * 64 + j % 64) * 8 + i % 8
    bp[idx.ravel()] = codes.ravel().astype(np.uint8)
    return bp


def _walk_codes(codes):
    """The path the codes give from (n-1, m-1), or None if they do not reach the origin."""
    n, m = codes.shape
    i, j = n - 1, m - 1
    out = [(i, j)]
    while (i, j) != (0, 0):
        c = int(codes[i, j])
        if c == 3:
            return None
        i, j = i - 1 - (c >> 1), j - 1 - (c & 1)
        if i < 0 or j < 0:
            return None
        out.append((i, j))
    return np.array(out[::-1], dtype=np.int32)


def _random_walk_codes(n, m, seed):
    """Codes drawn at random among the steps that stay in the cone of cells
    the origin reaches (i <= 2j, j <= 2i), 3 at the origin: the walk from any
    cone cell reaches the origin, and the paths of nearby cells are unrelated
    random walks that seldom merge."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)[:, None]
    j = np.arange(m)[None, :]

    def cone(a, b):
        return (a >= 0) & (b >= 0) & (a <= 2 * b) & (b <= 2 * a)

    ok = np.stack([cone(i - 1, j - 1), cone(i - 1, j - 2), cone(i - 2, j - 1)])  # codes 0, 1, 2
    first = rng.integers(0, 3, size=(n, m))
    codes = np.zeros((n, m), dtype=np.int8)
    chosen = np.zeros((n, m), dtype=bool)
    for t in range(3):  # the first allowed code from a random one on, cyclically
        c = (first + t) % 3
        take = ~chosen & np.take_along_axis(ok, c[None], 0)[0]
        codes[take] = c[take]
        chosen |= take
    codes[0, 0] = 3
    return codes


@pytest.mark.parametrize("n,m,seed", [(3000, 3400, 11), (9000, 9500, 12)])
def test_split_walk_on_random_walk_codes(n, m, seed):
    codes = _random_walk_codes(n, m, seed)
    ref = _walk_codes(codes)
    assert ref is not None and len(ref) <= min(n, m)
    bp = torch.from_numpy(_pack_bytes(codes)).to(DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ser, par = _paths(bp, n, m, st)
    assert np.array_equal(ser, ref)
    assert np.array_equal(par, ref)


@pytest.mark.parametrize("where", [0.1, 0.5, 0.93])
def test_split_walk_fails_on_corrupt_codes(where):
    """Code 3 planted on the path (away from the origin): both walks fail."""
    rng = np.random.default_rng(5)
    n, m = 4000, 4500
    X, Y = synth.chroma_like(rng, n), synth.chroma_like(rng, m)
    J, BP = oracle.dtw_features(X, Y)
    path = oracle.backtrace(BP)
    codes = BP.copy()
    ci, cj = path[int(where * (len(path) - 1))]
    codes[ci, cj] = 3
    bp = torch.from_numpy(_pack_bytes(codes)).to(DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    ser, par = _paths(bp, n, m, st)
    assert len(ser) == 0 and len(par) == 0
    # and without the planted code both give the oracle's path
    bp = torch.from_numpy(_pack_bytes(BP)).to(DEV)
    ser, par = _paths(bp, n, m, st)
    assert np.array_equal(ser, path) and np.array_equal(par, path)


def test_split_walk_infeasible_and_bad_arguments():
    n, m = 100, 400  # no path: m - 1 > 2 (n - 1)
    bp = torch.zeros(pd.pardtw_bp_bytes(n, m), dtype=torch.uint8, device=DEV)
    st = torch.full((1,), pd.PAIR_INFEASIBLE, dtype=torch.int32, device=DEV)
    ser, par = _paths(bp, n, m, st)
    assert len(ser) == 0 and len(par) == 0
    path = torch.empty((min(n, m), 2), dtype=torch.int32, device=DEV)
    plen = torch.empty(1, dtype=torch.int32, device=DEV)
    small = torch.empty(pd.pardtw_backtrace_parallel_bytes(n, m) - 16, dtype=torch.uint8, device=DEV)
    with pytest.raises(pd.PardtwError, match="ERR_WORKSPACE"):
        pd.pardtw_backtrace_parallel(bp, n, m, st, path, plen, small)


def test_split_walk_long_pair():
    """The 50000 x 60000 chroma pair: the split walk's path is the serial one's."""
    X, Y = synth.make_workload("pair_50000x60000_d12")
    n, m = len(X), len(Y)
    w = pd.Workspace(n, m, DEV, cost=False)
    pd.align_into(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), w, fused=True, serial_backtrace=True)
    ser, par = _paths(w.bp, n, m, w.status)
    assert len(ser) > 0 and np.array_equal(ser, par)
