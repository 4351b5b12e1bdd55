"""The DP with the cost computed inside it (the paper's on-the-fly cost, Sec.
II-D): bit for bit the materialised cost GEMM followed by the DP, and the
FP64 oracle's path and total, through the C ABI."""
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


def _run(X, Y, fused, sub=False, nw=0, layout=pd.LAYOUT_PANEL):
    n, m = X.shape[0], Y.shape[0]
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    bp = torch.empty(pd.pardtw_bp_bytes(n, m), dtype=torch.uint8, device=DEV)
    ws = torch.zeros(pd.pardtw_dp_workspace_bytes(n, m), dtype=torch.uint8, device=DEV)
    out = torch.empty(m if sub else 1, dtype=torch.float32, device=DEV)
    st = torch.empty(1, dtype=torch.int32, device=DEV)
    if fused:
        if sub:
            pd.pardtw_subseq_dp_fused(Xd, Yd, bp, out, st, ws)
        else:
            pd.pardtw_dp_fused(Xd, Yd, bp, out, st, ws, panels_per_workgroup=nw)
    else:
        C = torch.empty(pd.pardtw_cost_elems(n, m, layout), dtype=torch.float32, device=DEV)
        pd.pardtw_cost(Xd, Yd, C, pd.PREC_F32, layout)
        if sub:
            pd.pardtw_subseq_dp(C, n, m, bp, out, st, ws, layout)
        else:
            pd.pardtw_dp(C, n, m, bp, out, st, ws, layout, panels_per_workgroup=nw or None)
    B = pd.pardtw_bp_unpack(bp, n, m).cpu().numpy()
    path = np.empty((0, 2), np.int32)
    if not sub:
        p = torch.empty((min(n, m), 2), dtype=torch.int32, device=DEV)
        pl = torch.empty(1, dtype=torch.int32, device=DEV)
        pd.pardtw_backtrace(bp, n, m, st, p, pl)
        path = p[: int(pl.item())].cpu().numpy()
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.item()), B, path


def _features(seed, n, m, d):
    rng = np.random.default_rng(seed)
    X = synth.chroma_like(rng, n, d).astype(np.float32)
    Y = synth.chroma_like(rng, m, d).astype(np.float32)
    return X, Y


SHAPES = [(1, 1), (2, 3), (7, 5), (8, 8), (9, 17), (16, 20), (17, 30), (63, 64), (64, 65), (65, 100), (130, 170),
          (333, 400), (600, 520), (777, 1500), (1000, 1200), (100, 199), (100, 250)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("d", [12, 1, 5, 16])
def test_fused_dp_bit_identical_to_cost_then_dp(n, m, d):
    X, Y = _features(n * 31 + m + d, n, m, d)
    ref = _run(X, Y, fused=False, layout=pd.LAYOUT_PANEL_BAND)
    got = _run(X, Y, fused=True)
    band = parity.band_mask(n, m)
    assert got[1] == ref[1]
    assert got[0][0] == ref[0][0] or (np.isinf(got[0][0]) and np.isinf(ref[0][0]))
    assert np.array_equal(got[2][band], ref[2][band])
    assert np.array_equal(got[3], ref[3])


@pytest.mark.parametrize("nw", [1, 2, 4])
def test_fused_dp_schedules_identical(nw):
    X, Y = _features(3, 777, 1500, 12)
    ref = _run(X, Y, fused=False, nw=1)
    got = _run(X, Y, fused=True, nw=nw)
    band = parity.band_mask(777, 1500)
    assert got[0][0] == ref[0][0] and got[1] == ref[1]
    assert np.array_equal(got[2][band], ref[2][band]) and np.array_equal(got[3], ref[3])


@pytest.mark.parametrize("n,m", [(1, 70), (9, 5), (40, 17), (100, 3000), (333, 2100), (1562, 6000), (700, 300)])
def test_fused_subseq_bit_identical(n, m):
    X, Y = _features(n + 7 * m, n, m, 12)
    ref = _run(X, Y, fused=False, sub=True, layout=pd.LAYOUT_PANEL_SUBSEQ_BAND)
    got = _run(X, Y, fused=True, sub=True)
    band = parity.subseq_band_mask(n, m)
    assert got[1] == ref[1]
    assert np.array_equal(np.isinf(got[0]), np.isinf(ref[0]))
    fin = np.isfinite(ref[0])
    assert np.array_equal(got[0][fin], ref[0][fin])
    assert np.array_equal(got[2][band], ref[2][band])


def test_fused_zero_frames_and_unsupported_d():
    X, Y = _features(4, 200, 230, 12)
    X[0] = 0.0
    X[57] = 0.0
    Y[101] = 0.0
    ref = _run(X, Y, fused=False)
    got = _run(X, Y, fused=True)
    assert got[0][0] == ref[0][0] and np.array_equal(got[3], ref[3])
    Xd = torch.zeros((10, 17), dtype=torch.float32, device=DEV)
    Yd = torch.zeros((10, 17), dtype=torch.float32, device=DEV)
    bp = torch.empty(pd.pardtw_bp_bytes(10, 10), dtype=torch.uint8, device=DEV)
    ws = torch.zeros(pd.pardtw_dp_workspace_bytes(10, 10), dtype=torch.uint8, device=DEV)
    t = torch.empty(1, dtype=torch.float32, device=DEV)
    s = torch.empty(1, dtype=torch.int32, device=DEV)
    with pytest.raises(pd.PardtwError):
        pd.pardtw_dp_fused(Xd, Yd, bp, t, s, ws)


@pytest.mark.parametrize("n,m", [(1000, 1200), (2000, 2400)])
def test_fused_dp_against_oracle(n, m):
    X, Y = synth.chroma_pair(n + m, n, m)
    total, BP = oracle.dtw_features(X, Y)
    g_tot, g_st, _, g_path = _run(X, Y, fused=True)
    assert g_st == pd.PAIR_OK
    parity.check_total(float(g_tot[0]), total)
    parity.check_legal(g_path, n, m)
    parity.audit_path(g_path, BP, lambda c: oracle.probe(c, X=X, Y=Y)[0])


@pytest.mark.slow
def test_fused_full_size_identical():
    """50000 x 60000: the fused DP against cost + DP, total and path."""
    X, Y = synth.make_workload("pair_50000x60000_d12")
    n, m = X.shape[0], Y.shape[0]
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    res = []
    for fused in (False, True):
        w = pd.Workspace(n, m, DEV, pd.LAYOUT_PANEL_BAND, cost=not fused)
        pd.align_into(Xd, Yd, w, fused=fused)
        torch.cuda.synchronize()
        L = int(w.path_len.item())
        res.append((float(w.total.item()), w.path[:L].cpu().numpy()))
        del w
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
