"""The allocation-free DP entry point, pardtw_dp_noalloc, against pardtw_dp.

It takes no workspace argument: the library's static device array serves as
workspace. Two calls in a row (the second on a smaller pair, in another
layout, over the first call's leftover records), then an infeasible pair,
must each give pardtw_dp's codes on the path band, total bits, status and
backtraced path; a pair whose workspace exceeds the array is refused."""
import numpy as np
import pytest

from paper_2607_15478_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_15478_amd import pardtw as pd  # noqa: E402

DEV = "cuda:0"


def _dp_both(X, Y, layout):
    n, m = X.shape[0], Y.shape[0]
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
    C = torch.empty(pd.pardtw_cost_elems(n, m, layout), dtype=torch.float32, device=DEV)
    pd.pardtw_cost(Xd, Yd, C, pd.PREC_F32, layout)
    out = []
    for noalloc in (False, True):
        bp = torch.full((pd.pardtw_bp_bytes(n, m),), 0xAB, dtype=torch.uint8, device=DEV)
        total = torch.empty(1, dtype=torch.float32, device=DEV)
        status = torch.empty(1, dtype=torch.int32, device=DEV)
        path = torch.empty((min(n, m), 2), dtype=torch.int32, device=DEV)
        plen = torch.empty(1, dtype=torch.int32, device=DEV)
        if noalloc:
            pd.pardtw_dp_noalloc(C, n, m, bp, total, status, layout)
        else:
            ws = torch.zeros(pd.pardtw_dp_workspace_bytes(n, m), dtype=torch.uint8, device=DEV)
            pd.pardtw_dp(C, n, m, bp, total, status, ws, layout)
        pd.pardtw_backtrace(bp, n, m, status, path, plen)
        codes = pd.pardtw_bp_unpack(bp, n, m)
        torch.cuda.synchronize()
        L = int(plen.item())
        out.append(dict(total=total.cpu().numpy().view(np.uint32)[0], status=int(status.item()),
                        codes=codes.cpu().numpy(), path=path[:L].cpu().numpy()))
    return out


@pytest.mark.parametrize("n,m,layout,seed", [(3000, 3500, pd.LAYOUT_PANEL_BAND, 1), (700, 640, pd.LAYOUT_PANEL, 2),
                                             (90, 400, pd.LAYOUT_ROW, 3)])
def test_noalloc_matches_pardtw_dp(n, m, layout, seed):
    if oracle_feasible(n, m):
        X, Y = synth.chroma_pair(seed, n, m)
    else:
        rng = np.random.default_rng(seed)
        X, Y = synth.chroma_like(rng, n), synth.chroma_like(rng, m)
    ref, got = _dp_both(X, Y, layout)
    assert got["status"] == ref["status"]
    assert got["total"] == ref["total"]
    band = parity.band_mask(n, m)
    assert np.array_equal(got["codes"][band], ref["codes"][band])
    assert np.array_equal(got["path"], ref["path"])
    if not oracle_feasible(n, m):
        assert got["status"] == pd.PAIR_INFEASIBLE and len(got["path"]) == 0


def oracle_feasible(n, m):
    return (m - 1) <= 2 * (n - 1) and (n - 1) <= 2 * (m - 1)


def test_noalloc_refuses_pairs_past_its_array():
    n, m = 50000, 60000
    assert pd.pardtw_dp_workspace_bytes(n, m) > pd.NOALLOC_SCRATCH_BYTES
    C = torch.empty(pd.pardtw_cost_elems(n, m, pd.LAYOUT_PANEL_BAND), dtype=torch.float32, device=DEV)
    bp = torch.empty(pd.pardtw_bp_bytes(n, m), dtype=torch.uint8, device=DEV)
    total = torch.empty(1, dtype=torch.float32, device=DEV)
    status = torch.empty(1, dtype=torch.int32, device=DEV)
    with pytest.raises(pd.PardtwError, match="ERR_WORKSPACE"):
        pd.pardtw_dp_noalloc(C, n, m, bp, total, status, pd.LAYOUT_PANEL_BAND)
    # the largest square pair that fits still runs
    k = 15000
    assert pd.pardtw_dp_workspace_bytes(k, k) <= pd.NOALLOC_SCRATCH_BYTES
