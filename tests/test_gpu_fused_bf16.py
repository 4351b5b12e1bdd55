"""The fused cost with BF16 operands (plans with PARDTW_PLAN_FUSED_COST and
PARDTW_PREC_BF16, d <= 128, d % 8 == 0): the DP's producer waves run the cost
GEMM's own BF16 slab (panel operands, row operands, MFMA steps and their
order), so every total, status, code and path must equal those of the plan
that materialises the BF16 cost matrix, bit for bit, under every schedule,
and for Segmental DTW plans too."""
import numpy as np
import pytest

from paper_2607_15478_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_15478_amd import pardtw as pd  # noqa: E402

DEV = "cuda:0"


def _outputs(plan, buf):
    torch.cuda.synchronize()
    return (buf["totals"].cpu().numpy().copy(), buf["status"].cpu().numpy().copy(),
            buf["path_len"].cpu().numpy().copy(),
            [plan.path(buf, b).cpu().numpy().copy() for b in range(plan.batch)])


def _pairs(rng, shapes, d):
    out = []
    for n, m in shapes:
        if min(n, m) < 8 or (m - 1) > 2 * (n - 1) or (n - 1) > 2 * (m - 1):
            out.append((rng.standard_normal((n, d)).astype(np.float32),
                        rng.standard_normal((m, d)).astype(np.float32)))
        else:
            r = (m - 1) / (n - 1)
            out.append(synth.gaussian_pair(rng, n, m, d, 0.8 * r, 1.25 * r))
    return out


SHAPES = [(300, 350), (1000, 800), (64, 100), (2, 3), (5, 20), (1500, 2100), (17, 9), (2500, 2200), (700, 1400)]


@pytest.mark.parametrize("d", [8, 40, 64, 128])
def test_fused_bf16_plan_bit_identical(d):
    rng = np.random.default_rng(d)
    pairs = _pairs(rng, SHAPES, d)
    ns, ms = [p[0].shape[0] for p in pairs], [p[1].shape[0] for p in pairs]
    Xp, Yp = pd.pack(pairs, DEV)
    plan = pd.Plan(ns, ms, d, pd.PREC_BF16)
    buf = plan.buffers(DEV)
    plan.align(Xp, Yp, buf)
    ref = _outputs(plan, buf)
    assert (ref[1] == pd.PAIR_OK).sum() >= 6
    fplan = pd.Plan(ns, ms, d, pd.PREC_BF16, fused=True)
    fbuf = fplan.buffers(DEV)
    assert fplan.workspace_bytes < plan.workspace_bytes  # no cost matrix
    for s in range(fplan.num_schedules):
        fplan.select(s)
        assert fplan.schedule()["panels_per_workgroup"] <= 2
        fbuf["path_len"].fill_(-3)
        fplan.align(Xp, Yp, fbuf)
        got = _outputs(fplan, fbuf)
        assert np.array_equal(got[0].view(np.uint32), ref[0].view(np.uint32)), s
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
        for b in range(plan.batch):
            assert np.array_equal(got[3][b], ref[3][b]), (s, b)
    assert fplan.autotune(Xp, Yp, fbuf, reps=1) > 0


def test_fused_bf16_workload_shape():
    """The 32-pair, 2000-4000-frame, D = 128 workload itself: fused equals materialised."""
    pairs = synth.make_workload("batch32_2000to4000_d128")
    ns, ms = [len(p[0]) for p in pairs], [len(p[1]) for p in pairs]
    Xp, Yp = pd.pack(pairs, DEV)
    res = []
    for fused in (False, True):
        plan = pd.Plan(ns, ms, 128, pd.PREC_BF16, fused=fused)
        buf = plan.buffers(DEV)
        plan.align(Xp, Yp, buf)
        res.append(_outputs(plan, buf))
    (t0, s0, l0, p0), (t1, s1, l1, p1) = res
    assert np.array_equal(t0.view(np.uint32), t1.view(np.uint32))
    assert np.array_equal(s0, s1) and np.array_equal(l0, l1)
    assert all(np.array_equal(a, b) for a, b in zip(p0, p1))


def test_fused_bf16_unsupported_shapes():
    for d in (12, 136, 4):
        with pytest.raises(pd.PardtwError, match="UNSUPPORTED"):
            pd.Plan([100], [120], d, pd.PREC_BF16, fused=True)


@pytest.mark.parametrize("variant", [pd.NSDTW, pd.WSDTW])
def test_segmental_fused_bf16_bit_identical(variant):
    rng = np.random.default_rng(31)
    la, lb, nf, d = 2000, 2400, 8, 64
    A, B = synth.gaussian_pair(rng, la, lb, d, 0.8 * (lb - 1) / (la - 1), 1.25 * (lb - 1) / (la - 1))
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    outs = []
    for fused in (False, True):
        plan = pd.SegPlan(la, lb, nf, d, pd.PREC_BF16, variant, fused)
        buf = plan.buffers(DEV)
        plan.align(Ad, Bd, buf)
        torch.cuda.synchronize()
        L = int(buf["path_len"].item())
        outs.append((np.float32(buf["total"].item()).view(np.uint32), int(buf["status"].item()),
                     buf["ends"].cpu().numpy(), buf["path"][:L].cpu().numpy()))
    (t0, s0, e0, p0), (t1, s1, e1, p1) = outs
    assert s0 == s1 == pd.PAIR_OK and t0 == t1
    assert np.array_equal(e0, e1) and np.array_equal(p0, p1)
