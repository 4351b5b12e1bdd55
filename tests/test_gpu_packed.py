"""Packed 2-bit codes (Sec. VI-D's 2-bit transition types) against the byte
codes and the oracle.

The packed DP runs the same sweep and arithmetic as the byte-code DP, so on
the path band its codes, total and status must equal the byte codes' bit for
bit, for the materialised cost and the fused cost, and the packed backtrace
must return the same path. Small-integer costs make every sum exact, so there
the packed codes must also equal the FP64 oracle's codes on the band."""
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


def _run(X, Y, fused, packed, layout=pd.LAYOUT_PANEL_BAND):
    n, m = len(X), len(Y)
    w = pd.Workspace(n, m, DEV, layout, cost=not fused, packed=packed)
    w.bp.fill_(0xAB)
    pd.align_into(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), w, fused=fused)
    codes = pd.pardtw_bp2_unpack(w.bp, n, m) if packed else pd.pardtw_bp_unpack(w.bp, n, m)
    torch.cuda.synchronize()
    L = int(w.path_len.item())
    return dict(total=np.float32(w.total.item()).view(np.uint32), status=int(w.status.item()),
                codes=codes.cpu().numpy(), path=w.path[:L].cpu().numpy())


SHAPES = [(1, 1), (2, 3), (9, 17), (64, 65), (100, 199), (100, 200), (333, 400), (600, 520), (1000, 1200),
          (777, 1500), (3000, 2600)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("fused", [False, True])
def test_packed_equals_byte_codes(n, m, fused):
    rng = np.random.default_rng(n * 7 + m)
    X, Y = synth.chroma_like(rng, n), synth.chroma_like(rng, m)
    ref = _run(X, Y, fused, packed=False)
    got = _run(X, Y, fused, packed=True)
    band = parity.band_mask(n, m)
    assert got["status"] == ref["status"] and got["total"] == ref["total"]
    assert np.array_equal(got["codes"][band], ref["codes"][band])
    assert np.array_equal(got["path"], ref["path"])


@pytest.mark.parametrize("n,m", [(8, 8), (40, 50), (130, 170), (500, 700), (1300, 1100)])
def test_packed_integer_costs_match_the_oracle(n, m):
    """Small-integer cost matrices (exact sums): the packed DP's band codes are
    the oracle's, and the packed backtrace its path."""
    rng = np.random.default_rng(n + 11 * m)
    C = rng.integers(0, 3, size=(n, m)).astype(np.float32)
    J, BP, _ = oracle.dtw_matrix(C)
    Cd = torch.from_numpy(parity.to_panel(C)).to(DEV)
    bp2 = torch.empty(pd.pardtw_bp2_bytes(n, m), dtype=torch.uint8, device=DEV)
    ws = torch.zeros(pd.pardtw_dp_workspace_bytes(n, m), dtype=torch.uint8, device=DEV)
    total = torch.empty(1, dtype=torch.float32, device=DEV)
    st = torch.empty(1, dtype=torch.int32, device=DEV)
    path = torch.empty((min(n, m), 2), dtype=torch.int32, device=DEV)
    plen = torch.empty(1, dtype=torch.int32, device=DEV)
    pd.pardtw_dp_packed(Cd, n, m, bp2, total, st, ws, pd.LAYOUT_PANEL)
    pd.pardtw_backtrace_packed(bp2, n, m, st, path, plen)
    B = pd.pardtw_bp2_unpack(bp2, n, m).cpu().numpy()
    torch.cuda.synchronize()
    band = parity.band_mask(n, m)
    assert np.array_equal(B[band], BP[band])
    assert float(total.item()) == J
    assert np.array_equal(path[: int(plen.item())].cpu().numpy(), oracle.backtrace(BP))


def test_packed_long_pair_against_the_oracle():
    """A 10000 x 12000 chroma pair with the fused packed DP: legal path, the
    oracle's up to declared ties, total within 1e-5."""
    X, Y = synth.make_workload("pair_10000x12000_d12")
    got = _run(X, Y, fused=True, packed=True)
    J, BP = oracle.dtw_features(X, Y)
    parity.check_legal(got["path"], len(X), len(Y))
    parity.check_total(float(got["total"].view(np.float32)), J)
    parity.audit_path(got["path"], BP, lambda c: oracle.probe(c, X=X, Y=Y)[0])


def test_packed_bytes_and_bad_arguments():
    n, m = 50000, 60000
    assert pd.pardtw_bp2_bytes(n, m) * 4 == pd.pardtw_bp_bytes(n, m)
    C = torch.empty(pd.pardtw_cost_elems(10, 12, pd.LAYOUT_ROW), dtype=torch.float32, device=DEV)
    bp2 = torch.empty(pd.pardtw_bp2_bytes(10, 12), dtype=torch.uint8, device=DEV)
    ws = torch.zeros(pd.pardtw_dp_workspace_bytes(10, 12), dtype=torch.uint8, device=DEV)
    t = torch.empty(1, dtype=torch.float32, device=DEV)
    st = torch.empty(1, dtype=torch.int32, device=DEV)
    with pytest.raises(pd.PardtwError, match="UNSUPPORTED"):
        pd.pardtw_dp_packed(C, 10, 12, bp2, t, st, ws, pd.LAYOUT_ROW)
