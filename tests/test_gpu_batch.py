"""Batched form (pardtw_plan_* / pardtw_align_batch) on the GPU.

The batch runs the same cost, DP and backtrace code as the single-pair entry
points, so every pair's total and path must be bit-identical to a single-pair
call, whatever schedule the plan uses, and must pass the oracle parity rules.
"""
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
SHAPES = [(1, 1), (2, 3), (3, 2), (5, 20), (64, 65), (300, 129), (500, 700), (700, 500), (130, 64), (1200, 1000),
          (2000, 1500), (1000, 3000), (1500, 2900), (17, 9), (900, 901)]


def _pair(rng, n, m, d=12):
    if min(n, m) < 8:
        x = rng.random((n, d), dtype=np.float32) + 0.05
        y = rng.random((m, d), dtype=np.float32) + 0.05
        return x, y
    r = (m - 1) / (n - 1)
    return synth.chroma_pair(rng, n, m, d, 0.8 * r, 1.25 * r)


@pytest.fixture(scope="module")
def mixed():
    rng = np.random.default_rng(11)
    pairs = [_pair(rng, n, m) for n, m in SHAPES]
    plan = pd.Plan([p[0].shape[0] for p in pairs], [p[1].shape[0] for p in pairs], 12)
    Xp, Yp = pd.pack(pairs, DEV)
    buf = plan.buffers(DEV)
    plan.align(Xp, Yp, buf)
    torch.cuda.synchronize()
    return pairs, plan, Xp, Yp, buf


def _single(x, y, prec=pd.PREC_F32):
    w = pd.Workspace(len(x), len(y), DEV)
    pd.align_into(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV), w, prec)
    torch.cuda.synchronize()
    L = int(w.path_len.item())
    return float(w.total.item()), int(w.status.item()), w.path[:L].cpu().numpy()


def _outputs(plan, buf):
    torch.cuda.synchronize()
    return (buf["totals"].cpu().numpy().copy(), buf["status"].cpu().numpy().copy(),
            buf["path_len"].cpu().numpy().copy(),
            [plan.path(buf, b).cpu().numpy().copy() for b in range(plan.batch)])


def test_batch_matches_single_pair_and_oracle(mixed):
    pairs, plan, _, _, buf = mixed
    totals, status, plen, paths = _outputs(plan, buf)
    for b, (x, y) in enumerate(pairs):
        n, m = len(x), len(y)
        if not oracle.feasible(n, m):
            assert status[b] == pd.PAIR_INFEASIBLE and np.isinf(totals[b]) and plen[b] == 0
            continue
        t1, s1, p1 = _single(x, y)
        assert status[b] == pd.PAIR_OK == s1
        assert totals[b] == np.float32(t1) and np.array_equal(paths[b], p1), (n, m)
        J, BP = oracle.dtw_features(x, y)
        parity.check_legal(paths[b], n, m)
        parity.check_total(float(totals[b]), J)
        parity.audit_path(paths[b], BP, lambda c: oracle.probe(c, X=x, Y=y)[0])


def test_every_schedule_is_bit_identical(mixed):
    pairs, plan, Xp, Yp, buf = mixed
    ref = _outputs(plan, buf)
    default = plan.selected
    assert plan.num_schedules >= 8
    try:
        for s in range(plan.num_schedules):
            plan.select(s)
            buf["paths"].fill_(-1)
            buf["totals"].fill_(-1)
            plan.align(Xp, Yp, buf)
            got = _outputs(plan, buf)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), plan.schedule(s)
            assert np.array_equal(got[2], ref[2])
            assert all(np.array_equal(a, c) for a, c in zip(got[3], ref[3])), plan.schedule(s)
    finally:
        plan.select(default)


def test_autotune_selects_a_schedule_and_keeps_results(mixed):
    pairs, plan, Xp, Yp, buf = mixed
    ref = _outputs(plan, buf)
    best = plan.autotune(Xp, Yp, buf, reps=1)
    assert best > 0 and 0 <= plan.selected < plan.num_schedules
    plan.align(Xp, Yp, buf)
    got = _outputs(plan, buf)
    assert np.array_equal(got[0], ref[0]) and all(np.array_equal(a, c) for a, c in zip(got[3], ref[3]))


def test_graph_capture_replays_match_eager(mixed):
    pairs, plan, Xp, Yp, buf = mixed
    ref = _outputs(plan, buf)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.align(Xp, Yp, buf)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.align(Xp, Yp, buf)
    x0, y0 = pairs[8]
    for rep in range(3):
        # eager work between replays: clobber the outputs, run a single-pair call
        buf["paths"].fill_(-5)
        buf["totals"].fill_(7.0)
        buf["path_len"].fill_(-1)
        buf["status"].fill_(9)
        _single(x0, y0)
        g.replay()
        got = _outputs(plan, buf)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), rep
        assert np.array_equal(got[2], ref[2]), rep
        assert all(np.array_equal(a, c) for a, c in zip(got[3], ref[3])), rep


def test_batch_gradient_matches_single_pair(mixed):
    pairs, plan, Xp, Yp, buf = mixed
    g = torch.linspace(0.5, 2.0, plan.batch, device=DEV)
    dX = torch.full_like(Xp, 3.0)
    dY = torch.full_like(Yp, 3.0)
    plan.path_grad(Xp, Yp, buf, g, dX, dY)
    torch.cuda.synchronize()
    for b, (x, y) in enumerate(pairs):
        xs, ys = slice(plan.x_off[b], plan.x_off[b] + len(x)), slice(plan.y_off[b], plan.y_off[b] + len(y))
        if not oracle.feasible(len(x), len(y)):
            assert torch.count_nonzero(dX[xs]) == 0 and torch.count_nonzero(dY[ys]) == 0
            continue
        path = plan.path(buf, b).contiguous()
        plen = torch.tensor([len(path)], dtype=torch.int32, device=DEV)
        dx1 = torch.empty((len(x), 12), device=DEV)
        dy1 = torch.empty((len(y), 12), device=DEV)
        pd.pardtw_path_grad(Xp[xs].contiguous(), Yp[ys].contiguous(), path, plen, g[b:b + 1].contiguous(), dx1, dy1)
        torch.cuda.synchronize()
        assert torch.equal(dX[xs], dx1) and torch.equal(dY[ys], dy1), b
        if b in (6, 9):
            gx, gy = oracle.path_grad(x, y, path.cpu().numpy(), float(g[b]))
            np.testing.assert_allclose(dx1.cpu().numpy(), gx, rtol=1e-4, atol=1e-5)
            np.testing.assert_allclose(dy1.cpu().numpy(), gy, rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("prec", [pd.PREC_BF16, pd.PREC_F32])
def test_batch_d128_matches_single_pair(prec):
    rng = np.random.default_rng(5)
    shapes = [(300, 350), (1000, 800), (64, 100)]
    pairs = [synth.gaussian_pair(rng, n, m, 128, 0.8 * (m - 1) / (n - 1), 1.25 * (m - 1) / (n - 1))
             for n, m in shapes]
    plan = pd.Plan([n for n, _ in shapes], [m for _, m in shapes], 128, prec)
    Xp, Yp = pd.pack(pairs, DEV)
    buf = plan.buffers(DEV)
    plan.align(Xp, Yp, buf)
    totals, status, _, paths = _outputs(plan, buf)
    for b, (x, y) in enumerate(pairs):
        t1, s1, p1 = _single(x, y, prec)
        assert totals[b] == np.float32(t1) and np.array_equal(paths[b], p1)


def test_batch_workload_sample_against_oracle():
    """The first 16 pairs of the 256-pair chroma batch (lengths 500..8000)."""
    pairs = synth.make_workload("batch256_500to8000_d12")[:16]
    plan = pd.Plan([len(p[0]) for p in pairs], [len(p[1]) for p in pairs], 12)
    Xp, Yp = pd.pack(pairs, DEV)
    buf = plan.buffers(DEV)
    plan.align(Xp, Yp, buf)
    totals, status, plen, paths = _outputs(plan, buf)
    for b, (x, y) in enumerate(pairs):
        n, m = len(x), len(y)
        if not oracle.feasible(n, m):
            assert status[b] == pd.PAIR_INFEASIBLE and plen[b] == 0
            continue
        J, BP = oracle.dtw_features(x, y)
        parity.check_legal(paths[b], n, m)
        parity.check_total(float(totals[b]), J)
        parity.audit_path(paths[b], BP, lambda c: oracle.probe(c, X=x, Y=y)[0])


def test_fused_plan_bit_identical(mixed):
    """A plan whose DP computes the costs itself gives every pair the unfused
    plan's total, status and path, under each of its schedules."""
    pairs, plan, Xp, Yp, buf = mixed
    ref = _outputs(plan, buf)
    fplan = pd.Plan([p[0].shape[0] for p in pairs], [p[1].shape[0] for p in pairs], 12, fused=True)
    fbuf = fplan.buffers(DEV)
    assert fplan.workspace_bytes < plan.workspace_bytes  # no cost matrix
    for s in range(fplan.num_schedules):
        fplan.select(s)
        assert fplan.schedule()["panels_per_workgroup"] <= 4
        fplan.align(Xp, Yp, fbuf)
        got = _outputs(fplan, fbuf)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
        for b in range(plan.batch):
            assert np.array_equal(got[3][b], ref[3][b]), (s, b)
    assert fplan.autotune(Xp, Yp, fbuf, reps=1) > 0
    with pytest.raises(pd.PardtwError):
        pd.Plan([10], [10], 17, fused=True)
    with pytest.raises(pd.PardtwError):
        pd.Plan([10], [10], 12, pd.PREC_BF16, fused=True)


def test_split_walks_of_long_pairs_equal_the_serial_walk():
    """Pairs of more than 1024 rows are walked by the split walk inside the
    batch. Uniform random frames make nearby optimal paths merge slowly, so
    guessed segment starts miss and the final check walks segments again:
    every path must still equal the one-workgroup walk's."""
    rng = np.random.default_rng(23)
    shapes = [(2500, 2700), (4100, 3500), (1025, 1500), (5000, 5000), (900, 1000), (3000, 2000)]
    pairs = [(rng.random((n, 12), dtype=np.float32), rng.random((m, 12), dtype=np.float32)) for n, m in shapes]
    plan = pd.Plan([n for n, _ in shapes], [m for _, m in shapes], 12)
    Xp, Yp = pd.pack(pairs, DEV)
    buf = plan.buffers(DEV)
    plan.align(Xp, Yp, buf)
    totals, status, plen, paths = _outputs(plan, buf)
    for b, (x, y) in enumerate(pairs):
        w = pd.Workspace(len(x), len(y), DEV)
        pd.align_into(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV), w, serial_backtrace=True)
        torch.cuda.synchronize()
        L = int(w.path_len.item())
        assert L > 0 and plen[b] == L
        assert np.array_equal(paths[b], w.path[:L].cpu().numpy())
        assert np.float32(totals[b]) == np.float32(w.total.item())
