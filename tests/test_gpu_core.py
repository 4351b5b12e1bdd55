"""GPU parity of the single-pair hot path (cost, DP, backtrace, gradient)
against the FP64 oracle, through the C ABI."""

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


def _gpu_dp(C: np.ndarray, layout=pd.LAYOUT_ROW, nw=None):
    n, m = C.shape
    Cd = torch.from_numpy(parity.to_panel(C) if layout == pd.LAYOUT_PANEL else C.reshape(-1).copy()).to(DEV)
    bp = torch.empty(pd.pardtw_bp_bytes(n, m), dtype=torch.uint8, device=DEV)
    ws = torch.zeros(pd.pardtw_dp_workspace_bytes(n, m), dtype=torch.uint8, device=DEV)
    total = torch.empty(1, dtype=torch.float32, device=DEV)
    status = torch.empty(1, dtype=torch.int32, device=DEV)
    pd.pardtw_dp(Cd, n, m, bp, total, status, ws, layout, panels_per_workgroup=nw)
    B = pd.pardtw_bp_unpack(bp, n, m)
    path = torch.empty((min(n, m), 2), dtype=torch.int32, device=DEV)
    plen = torch.empty(1, dtype=torch.int32, device=DEV)
    pd.pardtw_backtrace(bp, n, m, status, path, plen)
    torch.cuda.synchronize()
    L = int(plen.item())
    return (float(total.item()), int(status.item()), B.cpu().numpy(), path[:L].cpu().numpy())


SHAPES = [(1, 1), (2, 2), (2, 3), (3, 2), (4, 4), (5, 9), (9, 5), (7, 1), (1, 7), (8, 8), (63, 64), (64, 65),
          (65, 63), (64, 127), (127, 64), (100, 199), (100, 200), (129, 300), (300, 129), (257, 513),
          (333, 400), (520, 700), (700, 520)]


@pytest.mark.parametrize("n,m", SHAPES)
def test_dp_integer_costs_bit_exact(n, m):
    """Small-integer costs: every sum is exact in FP32 and FP64, so the codes
    of every cell that can lie on a path (the band), the total and the path
    must match bit for bit, including the tie rule."""
    rng = np.random.default_rng(n * 1000 + m)
    C = rng.integers(0, 3, size=(n, m)).astype(np.float32)
    total, BP, _ = oracle.dtw_matrix(C)
    g_total, g_status, g_BP, g_path = _gpu_dp(C)
    band = parity.band_mask(n, m)
    assert np.array_equal(g_BP[band], BP[band])
    # band cells are reachable: the oracle gives them a real step, the origin code 3
    inner = band.copy()
    inner[0, 0] = False
    assert np.all(BP[inner] <= 2) and (not band[0, 0] or BP[0, 0] == 3)
    if oracle.feasible(n, m):
        assert g_status == pd.PAIR_OK and g_total == total
        assert np.array_equal(g_path, oracle.backtrace(BP))
    else:
        assert g_status == pd.PAIR_INFEASIBLE and np.isinf(g_total) and len(g_path) == 0


@pytest.mark.parametrize("c", [0.5, 1.0])
@pytest.mark.parametrize("n,m", [(200, 260), (260, 200), (129, 257), (1000, 1200)])
def test_dp_constant_cost_closed_form(c, n, m):
    C = np.full((n, m), c, dtype=np.float32)
    g_total, g_status, g_BP, g_path = _gpu_dp(C)
    assert g_total == c * (n + m - 1)
    codes = parity.step_codes(g_path).tolist()
    if n <= m:
        assert codes == [1] * (m - n) + [0] * (2 * n - m - 1)
    else:
        assert codes == [2] * (n - m) + [0] * (2 * m - n - 1)


@pytest.mark.parametrize("n,m", [(130, 170), (333, 400), (600, 520), (1000, 1200)])
def test_dp_random_costs_full_bp(n, m):
    rng = np.random.default_rng(7 + n)
    C = rng.uniform(0.0, 1.0, size=(n, m)).astype(np.float32)
    total, BP, D = oracle.dtw_matrix(C, want_D=True)
    g_total, g_status, g_BP, g_path = _gpu_dp(C)
    band = parity.band_mask(n, m)
    g_BP = np.where(band, g_BP, BP)  # codes outside the band are unspecified
    ties = parity.audit_bp_matrix(g_BP, BP, D, C)
    assert ties <= 1e-4 * n * m + 5
    parity.check_total(g_total, total)
    parity.check_legal(g_path, n, m)


@pytest.mark.parametrize("nw", [1, 2, 4])
def test_dp_schedules_and_layouts_bit_identical(nw):
    rng = np.random.default_rng(99)
    n, m = 777, 1500  # 24 panels, ragged last panel and last row group
    C = rng.uniform(0.0, 1.0, size=(n, m)).astype(np.float32)
    ref = _gpu_dp(C, pd.LAYOUT_ROW, nw=1)
    band = parity.band_mask(n, m)
    for layout in (pd.LAYOUT_ROW, pd.LAYOUT_PANEL):
        got = _gpu_dp(C, layout, nw=nw)
        assert got[0] == ref[0] and got[1] == ref[1]
        assert np.array_equal(got[2][band], ref[2][band]) and np.array_equal(got[3], ref[3])


def _gpu_cost(X, Y, prec=pd.PREC_F32, layout=pd.LAYOUT_ROW):
    n, m = X.shape[0], Y.shape[0]
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    C = torch.empty(pd.pardtw_cost_elems(n, m, layout), dtype=torch.float32, device=DEV)
    pd.pardtw_cost(Xd, Yd, C, prec, layout)
    c = C.cpu().numpy()
    return parity.from_panel(c, n, m) if layout == pd.LAYOUT_PANEL else c.reshape(n, m)


@pytest.mark.parametrize("n,m,d", [(1, 1, 12), (70, 130, 12), (333, 257, 12), (100, 90, 128), (65, 200, 5),
                                   (128, 64, 33),
                                   # the column operands held in registers (d <= 16), staged in LDS
                                   # (d a multiple of 16 up to 128) and loaded per tile (beyond):
                                   # several tiles per workgroup and a ragged last panel
                                   (600, 700, 16), (600, 700, 32), (257, 1000, 48), (1000, 300, 128),
                                   (600, 700, 144), (300, 333, 256)])
def test_cost_fp32_against_oracle(n, m, d):
    rng = np.random.default_rng(n + m + d)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Y = rng.normal(size=(m, d)).astype(np.float32)
    X[0] = 0.0  # a zero frame reads as the zero vector: cost 1
    ref = oracle.cost(X, Y)
    got_row = _gpu_cost(X, Y, pd.PREC_F32, pd.LAYOUT_ROW)
    got_pan = _gpu_cost(X, Y, pd.PREC_F32, pd.LAYOUT_PANEL)
    assert np.array_equal(got_row, got_pan)
    assert np.max(np.abs(got_row - ref)) < 4e-6 * max(1.0, np.sqrt(d / 12))
    assert np.all(got_row[0] == 1.0)


@pytest.mark.parametrize("n,m,d", [(100, 90, 128), (333, 257, 12), (64, 64, 40), (600, 700, 128),
                                   (600, 700, 136), (257, 1000, 16)])
def test_cost_bf16_against_oracle_on_rounded_inputs(n, m, d):
    rng = np.random.default_rng(n * m + d)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Y = rng.normal(size=(m, d)).astype(np.float32)
    ref = oracle.cost(parity.bf16_round(X), parity.bf16_round(Y))
    got = _gpu_cost(X, Y, pd.PREC_BF16, pd.LAYOUT_PANEL)
    assert np.max(np.abs(got - ref)) < 1e-5 * max(1.0, np.sqrt(d / 12))


@pytest.mark.parametrize("n,m,d,prec", [(1, 1, 12, pd.PREC_F32), (333, 257, 12, pd.PREC_F32),
                                        (700, 900, 12, pd.PREC_F32), (900, 700, 12, pd.PREC_F32),
                                        (1000, 130, 64, pd.PREC_F32), (600, 650, 33, pd.PREC_F32),
                                        (520, 700, 40, pd.PREC_BF16), (2000, 2400, 12, pd.PREC_F32),
                                        (1000, 1999, 12, pd.PREC_F32), (1999, 1000, 12, pd.PREC_F32),
                                        (3000, 2000, 12, pd.PREC_F32), (130, 1000, 12, pd.PREC_F32),
                                        (1000, 1300, 128, pd.PREC_F32), (1300, 1000, 32, pd.PREC_F32),
                                        (1000, 1300, 128, pd.PREC_BF16), (6000, 7000, 12, pd.PREC_F32),
                                        (7000, 3600, 12, pd.PREC_F32), (3600, 7000, 12, pd.PREC_F32)])
def test_cost_band_layout_writes_exactly_the_band_groups(n, m, d, prec):
    """The band layout holds the full panel layout's values bit for bit in
    every band group and leaves the others untouched; the larger shapes put
    the panels' first band groups in many different 512-row blocks, where the
    launch starts each panel's blocks."""
    rng = np.random.default_rng(n * 7 + m + d)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Y = rng.normal(size=(m, d)).astype(np.float32)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    full = torch.empty(pd.pardtw_cost_elems(n, m, pd.LAYOUT_PANEL), dtype=torch.float32, device=DEV)
    pd.pardtw_cost(Xd, Yd, full, prec, pd.LAYOUT_PANEL)
    part = torch.full((pd.pardtw_cost_elems(n, m, pd.LAYOUT_PANEL_BAND),), float("nan"), device=DEV)
    pd.pardtw_cost(Xd, Yd, part, prec, pd.LAYOUT_PANEL_BAND)
    P, G = -(-m // 64), -(-n // 8)
    f = full.cpu().numpy().reshape(P, G, 512)
    g = part.cpu().numpy().reshape(P, G, 512)
    written = parity.band_groups(n, m)
    assert np.array_equal(f[written], g[written])          # written groups: the panel layout bit for bit
    assert np.all(np.isnan(g[~written]))                    # the others untouched


@pytest.mark.parametrize("n,m", [(64, 65), (333, 400), (520, 700), (700, 520), (1500, 1300), (1000, 1999),
                                 (1999, 1000), (500, 1200)])
def test_dp_on_band_layout_matches_full_layout(n, m):
    rng = np.random.default_rng(n + 3 * m)
    X = rng.normal(size=(n, 12)).astype(np.float32)
    Y = rng.normal(size=(m, 12)).astype(np.float32)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    outs = []
    for layout in (pd.LAYOUT_PANEL, pd.LAYOUT_PANEL_BAND):
        w = pd.Workspace(n, m, DEV, layout)
        w.C.fill_(float("nan"))  # a read of an unwritten group would poison the result
        pd.align_into(Xd, Yd, w)
        B = pd.pardtw_bp_unpack(w.bp, n, m)
        torch.cuda.synchronize()
        L = int(w.path_len.item())
        outs.append((float(w.total.item()), int(w.status.item()), B.cpu().numpy(), w.path[:L].cpu().numpy()))
    a, b = outs
    band = parity.band_mask(n, m)
    assert a[0] == b[0] and a[1] == b[1]
    assert np.array_equal(a[2][band], b[2][band]) and np.array_equal(a[3], b[3])
    assert np.isfinite(a[0]) == oracle.feasible(n, m)
    if oracle.feasible(n, m):
        t_o, p_o, _ = oracle.align(X, Y)
        parity.check_total(a[0], t_o)
        parity.check_legal(a[3], n, m)
        assert np.all(band[a[3][:, 0], a[3][:, 1]])  # the path stays in the band


def _align(X, Y, prec=pd.PREC_F32):
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    total, path, status = pd.align(Xd, Yd, prec)
    return total, path.cpu().numpy(), status


@pytest.mark.parametrize("n,m,seed", [(1000, 1200, 1), (200, 150, 2), (300, 590, 3), (640, 641, 4)])
def test_align_end_to_end_against_oracle(n, m, seed):
    r = (m - 1) / (n - 1)
    if (n, m) == (1000, 1200):
        X, Y = synth.make_workload("pair_1000x1200_d12")
    else:
        X, Y = synth.chroma_pair(seed, n, m, lo=0.8 * r, hi=min(1.25 * r, 2.0))
    J, BP = oracle.dtw_features(X, Y)
    g_total, g_path, g_status = _align(X, Y)
    assert g_status == pd.PAIR_OK
    parity.check_legal(g_path, n, m)
    parity.check_total(g_total, J)
    parity.audit_path(g_path, BP, lambda cells: oracle.probe(cells, X=X, Y=Y)[0])
    assert oracle.path_cost(X, Y, g_path) <= J * (1 + 1e-6) + 1e-9


def test_align_infeasible_pair():
    X, Y = synth.chroma_pair(5, 100, 300, lo=2.5, hi=3.5)
    g_total, g_path, g_status = _align(X, Y)
    assert g_status == pd.PAIR_INFEASIBLE and np.isinf(g_total) and len(g_path) == 0


def test_self_alignment_diagonal():
    rng = np.random.default_rng(3)
    X = synth.chroma_like(rng, 700)
    g_total, g_path, g_status = _align(X, X)
    assert np.array_equal(g_path, np.stack([np.arange(700)] * 2, 1).astype(np.int32))
    assert abs(g_total) <= 2 * 700 * 1.2e-7 * 3


def test_path_grad_against_oracle():
    X, Y = synth.gaussian_pair(11, 300, 340, d=128, lo=0.8 * 339 / 299, hi=1.25 * 339 / 299)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    w = pd.Workspace(300, 340, DEV)
    pd.align_into(Xd, Yd, w)
    g = torch.tensor([0.75], dtype=torch.float32, device=DEV)
    dX = torch.full_like(Xd, 7.0)
    dY = torch.full_like(Yd, 7.0)
    pd.pardtw_path_grad(Xd, Yd, w.path, w.path_len, g, dX, dY)
    torch.cuda.synchronize()
    L = int(w.path_len.item())
    path = w.path[:L].cpu().numpy()
    rX, rY = oracle.path_grad(X, Y, path, 0.75)
    gx, gy = dX.cpu().numpy(), dY.cpu().numpy()
    scale = max(np.abs(rX).max(), np.abs(rY).max())
    assert np.max(np.abs(gx - rX)) <= 1e-5 * scale
    assert np.max(np.abs(gy - rY)) <= 1e-5 * scale
    skipped = np.setdiff1d(np.arange(300), path[:, 0])
    assert np.all(gx[skipped] == 0)


def test_align_10k_against_oracle():
    X, Y = synth.make_workload("pair_10000x12000_d12")
    J, BP = oracle.dtw_features(X, Y)
    g_total, g_path, g_status = _align(X, Y)
    parity.check_legal(g_path, 10000, 12000)
    parity.check_total(g_total, J)
    ties = parity.audit_path(g_path, BP, lambda cells: oracle.probe(cells, X=X, Y=Y)[0])
    print(f"10k x 12k: total {g_total} oracle {J} declared ties {ties}")


@pytest.mark.parametrize("n,m", [(333, 2100), (1500, 4000), (3000, 3100), (700, 9000), (2600, 1400)])
def test_cost_subseq_band_layout_writes_exactly_the_band_groups(n, m):
    """The subsequence band layout holds the full panel layout's values bit
    for bit in every group of the subsequence band (a cell that row 0 reaches
    and a cell that reaches row n-1, enumerated cell by cell) and leaves the
    others untouched, also where the panels' first band groups lie in
    different 512-row blocks."""
    rng = np.random.default_rng(n + 11 * m)
    X = rng.normal(size=(n, 12)).astype(np.float32)
    Y = rng.normal(size=(m, 12)).astype(np.float32)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    full = torch.empty(pd.pardtw_cost_elems(n, m, pd.LAYOUT_PANEL), dtype=torch.float32, device=DEV)
    pd.pardtw_cost(Xd, Yd, full, pd.PREC_F32, pd.LAYOUT_PANEL)
    part = torch.full((pd.pardtw_cost_elems(n, m, pd.LAYOUT_PANEL_SUBSEQ_BAND),), float("nan"), device=DEV)
    pd.pardtw_cost(Xd, Yd, part, pd.PREC_F32, pd.LAYOUT_PANEL_SUBSEQ_BAND)
    P, G = -(-m // 64), -(-n // 8)
    f = full.cpu().numpy().reshape(P, G, 512)
    g = part.cpu().numpy().reshape(P, G, 512)
    band = parity.subseq_band_groups(n, m)
    assert np.array_equal(f[band], g[band])
    assert np.all(np.isnan(g[~band]))
