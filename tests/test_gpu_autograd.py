"""Differentiable form (a6) and BF16-cost form (a7) on the GPU.

The gradient of J with the optimal path held fixed is checked against the FP64
oracle gradient, against central finite differences (eps = 1e-3) of the FP64
fixed-path total, and against finite differences of the full DTW wherever the
optimal path does not change under the perturbation (there the two agree)."""
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
from paper_2607_15478_amd.autograd import pardtw_batch_cost, pardtw_cost  # noqa: E402

DEV = "cuda:0"
EPS = 1e-3


def _pair(seed, n, m, d):
    r = (m - 1) / (n - 1)
    return synth.gaussian_pair(seed, n, m, d, 0.8 * r, 1.25 * r)


def _grads(x, y, g=1.0, prec=pd.PREC_F32):
    X = torch.from_numpy(x).to(DEV).requires_grad_(True)
    Y = torch.from_numpy(y).to(DEV).requires_grad_(True)
    total, path = pardtw_cost(X, Y, prec)
    (total * g).backward()
    return float(total.item()), path.cpu().numpy(), X.grad.cpu().numpy(), Y.grad.cpu().numpy()


def test_gradient_matches_fp64_oracle():
    x, y = _pair(21, 160, 190, 24)
    total, path, gx, gy = _grads(x, y, g=1.7)
    ox, oy = oracle.path_grad(x, y, path, 1.7)
    scale = max(np.abs(ox).max(), np.abs(oy).max())
    np.testing.assert_allclose(gx, ox, rtol=1e-4, atol=1e-5 * scale)
    np.testing.assert_allclose(gy, oy, rtol=1e-4, atol=1e-5 * scale)
    # rows and columns the path skips get exactly zero
    skipped = np.setdiff1d(np.arange(len(x)), path[:, 0])
    assert np.all(gx[skipped] == 0.0)


def test_gradient_matches_finite_differences():
    x, y = _pair(22, 60, 75, 8)
    _, path, gx, gy = _grads(x, y)
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    rng = np.random.default_rng(0)
    stable = 0
    for which, arr, grad in (("x", x64, gx), ("y", y64, gy)):
        for _ in range(24):
            r, c = int(rng.integers(arr.shape[0])), int(rng.integers(arr.shape[1]))
            plus, minus = arr.copy(), arr.copy()
            plus[r, c] += EPS
            minus[r, c] -= EPS
            xa, ya = (plus, y64) if which == "x" else (x64, plus)
            xb, yb = (minus, y64) if which == "x" else (x64, minus)
            # fixed-path total: smooth, its central difference is O(eps^2) from the derivative
            fd = (oracle.path_cost(xa, ya, path) - oracle.path_cost(xb, yb, path)) / (2 * EPS)
            assert abs(fd - grad[r, c]) <= 2e-3 * abs(fd) + 2e-4, (which, r, c, fd, grad[r, c])
            # full DTW (the path re-optimised): equal where the optimum does not move
            Ja, Ba = oracle.dtw_features(xa, ya)
            Jb, Bb = oracle.dtw_features(xb, yb)
            if np.array_equal(oracle.backtrace(Ba), path) and np.array_equal(oracle.backtrace(Bb), path):
                stable += 1
                assert abs((Ja - Jb) / (2 * EPS) - grad[r, c]) <= 2e-3 * abs(fd) + 2e-4
    assert stable >= 24  # most perturbations of size 1e-3 keep the optimal path


def test_autograd_composes_with_other_ops():
    x, y = _pair(23, 100, 90, 16)
    X = torch.from_numpy(x).to(DEV).requires_grad_(True)
    Y = torch.from_numpy(y).to(DEV).requires_grad_(True)
    total, _ = pardtw_cost(X, Y)
    loss = 2.0 * total + (X * X).sum()
    loss.backward()
    _, _, gx, gy = _grads(x, y, g=2.0)
    np.testing.assert_allclose(X.grad.cpu().numpy(), gx + 2.0 * x, rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(Y.grad.cpu().numpy(), gy)


def test_batch_autograd_matches_single_pairs():
    pairs = [_pair(30 + k, n, m, 32) for k, (n, m) in enumerate([(200, 230), (150, 120), (90, 170), (10, 40)])]
    plan = pd.Plan([len(p[0]) for p in pairs], [len(p[1]) for p in pairs], 32)
    Xp, Yp = pd.pack(pairs, DEV)
    Xp.requires_grad_(True)
    Yp.requires_grad_(True)
    buf = plan.buffers(DEV)
    totals = pardtw_batch_cost(Xp, Yp, plan, buf)
    w = torch.tensor([1.0, -0.5, 2.0, 3.0], device=DEV)
    (totals * w).sum().backward()
    for b, (x, y) in enumerate(pairs):
        xs = slice(plan.x_off[b], plan.x_off[b] + len(x))
        ys = slice(plan.y_off[b], plan.y_off[b] + len(y))
        if not oracle.feasible(len(x), len(y)):
            assert torch.count_nonzero(Xp.grad[xs]) == 0 and torch.isinf(totals[b])
            continue
        _, _, gx, gy = _grads(x, y, g=float(w[b]))
        np.testing.assert_array_equal(Xp.grad[xs].cpu().numpy(), gx)
        np.testing.assert_array_equal(Yp.grad[ys].cpu().numpy(), gy)


def test_bf16_cost_form_against_fp32_and_oracle():
    """The 32-pair D = 128 Gaussian workload, first 4 pairs: BF16-cost paths
    against the FP32 plain form (deviation in frames) and the FP64 optimum."""
    pairs = synth.make_workload("batch32_2000to4000_d128")[:4]
    ns, ms = [len(p[0]) for p in pairs], [len(p[1]) for p in pairs]
    Xp, Yp = pd.pack(pairs, DEV)
    out = {}
    for prec in (pd.PREC_F32, pd.PREC_BF16):
        plan = pd.Plan(ns, ms, 128, prec)
        buf = plan.buffers(DEV)
        plan.align(Xp, Yp, buf)
        torch.cuda.synchronize()
        out[prec] = (buf["totals"].cpu().numpy(), [plan.path(buf, b).cpu().numpy() for b in range(len(pairs))])
    report = []
    for b, (x, y) in enumerate(pairs):
        J, BP = oracle.dtw_features(x, y)
        p32, p16 = out[pd.PREC_F32][1][b], out[pd.PREC_BF16][1][b]
        parity.check_legal(p16, len(x), len(y))
        parity.check_total(float(out[pd.PREC_F32][0][b]), J)
        parity.audit_path(p32, BP, lambda c: oracle.probe(c, X=x, Y=y)[0])
        mean_dev, max_dev = parity.path_deviation(p16, p32, len(x))
        cost_err = abs(float(out[pd.PREC_BF16][0][b]) - J) / J
        gap = (oracle.path_cost(x, y, p16) - J) / J  # FP64 re-score of the BF16 path
        report.append((len(x), len(y), mean_dev, max_dev, cost_err, gap))
        # measured on this seeded workload: mean deviation 0.000 frames (max 1),
        # cost error <= 5.3e-5, re-score gap <= 1e-7; bounds keep a margin
        assert gap >= -1e-12 and gap < 1e-5 and mean_dev < 0.1 and max_dev <= 4 and cost_err < 1e-3
    print("\nBF16 cost form (n, m, mean dev, max dev [frames], |J_bf16 - J*|/J*, rescore gap):")
    for r in report:
        print("  %5d %5d %8.3f %6.1f %10.3e %10.3e" % r)
