"""GPU backtrace (pardtw_backtrace) on backtrace matrices with a known path.

The codes are written directly: a random legal path (runs of one step, so it
also follows the extreme slopes 1/2 and 2 for long stretches) gets its own
step codes and every other cell a random code. The walk reads only path cells,
so the result must be exactly the planted path; corrupt codes must give an
empty path, never a wrong one."""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_15478_amd import pardtw as pd  # noqa: E402

DEV = "cuda:0"


def _walk(B: np.ndarray, status: int = pd.PAIR_OK):
    n, m = B.shape
    bp = torch.from_numpy(parity.to_bp_layout(B)).to(DEV)
    assert bp.numel() == pd.pardtw_bp_bytes(n, m)
    st = torch.tensor([status], dtype=torch.int32, device=DEV)
    path = torch.full((min(n, m), 2), -7, dtype=torch.int32, device=DEV)
    plen = torch.empty(1, dtype=torch.int32, device=DEV)
    pd.pardtw_backtrace(bp, n, m, st, path, plen)
    torch.cuda.synchronize()
    L = int(plen.item())
    return path[:L].cpu().numpy()


SHAPES = [(1, 1), (2, 2), (2, 3), (3, 2), (5, 9), (9, 5), (64, 64), (65, 127), (127, 65), (130, 257),
          (200, 399), (399, 200), (1000, 1999), (1999, 1000), (1500, 1600), (3001, 2500), (4000, 7999),
          (7999, 4000), (6000, 9000), (9000, 6000)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("run", [3.0, 400.0])
def test_backtrace_planted_path(n, m, run):
    rng = np.random.default_rng(n * 7919 + m * 13 + int(run))
    path = parity.random_path(n, m, rng, mean_run=run)
    B = parity.bp_with_path(n, m, path, rng)
    got = _walk(B)
    assert got.shape == path.shape and np.array_equal(got, path)


def test_backtrace_infeasible_status_gives_empty_path():
    B = np.zeros((10, 30), dtype=np.uint8)
    assert len(_walk(B, status=pd.PAIR_INFEASIBLE)) == 0


@pytest.mark.parametrize("n,m", [(50, 60), (700, 500), (3000, 3300)])
def test_backtrace_corrupt_codes_give_empty_path(n, m):
    rng = np.random.default_rng(n + m)
    path = parity.random_path(n, m, rng)
    B = parity.bp_with_path(n, m, path, rng)
    k = len(path) // 2
    B[path[k, 0], path[k, 1]] = 3  # unreachable code in the middle of the path
    assert len(_walk(B)) == 0
    # all-diagonal codes on a non-square matrix run off the first row or column
    assert len(_walk(np.zeros((n, m), dtype=np.uint8))) == 0
