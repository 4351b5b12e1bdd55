"""The bench's pipelined schedule (each pair's backtrace on a backtrace
stream beside the next pairs' cost and DP, workspaces taken in turn): every
pair of the loop, not only the last, gets the result of the same pair
aligned on its own. Two layouts: two workspaces and one backtrace stream (the
default), three workspaces and two backtrace streams (checkpointed runs)."""
import numpy as np
import pytest

import bench
from paper_2607_15478_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_15478_amd import pardtw as pd  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("nbuf,nbt", [(2, 1), (3, 2)])
@pytest.mark.parametrize("mode", ["materialised", "fused", "ckpt"])
def test_every_pipelined_pair_matches_its_serial_alignment(mode, nbuf, nbt):
    n, m = 2000, 2400
    fused, K = mode == "fused", (64 if mode == "ckpt" else 0)
    X, Y = synth.chroma_pair(5, n, m)
    Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)

    def workspace():
        if K:
            return pd.Workspace(n, m, DEV, cost=False, ckpt_rows=K)
        return pd.Workspace(n, m, DEV, pd.LAYOUT_PANEL_BAND, cost=not fused)

    ref_w = workspace()
    pd.align_into(Xd, Yd, ref_w, fused=fused or bool(K))
    torch.cuda.synchronize()
    L = int(ref_w.path_len.item())
    ref_total, ref_path = float(ref_w.total.item()), ref_w.path[:L].cpu().numpy()

    steps = 7
    bufs = [workspace() for _ in range(nbuf)]
    for b in bufs:  # leave stale results from another pair in both workspaces
        X2, Y2 = synth.chroma_pair(6, n, m)
        pd.align_into(torch.from_numpy(X2).to(DEV), torch.from_numpy(Y2).to(DEV), b, fused=fused or bool(K))
    outs = [(torch.empty(1, device=DEV), torch.empty_like(bufs[0].path), torch.empty(1, dtype=torch.int32, device=DEV))
            for _ in range(steps)]

    def after_bt(s, w, s_bt):
        with torch.cuda.stream(s_bt):
            outs[s][0].copy_(w.total)
            outs[s][1].copy_(w.path)
            outs[s][2].copy_(w.path_len)

    stream = torch.cuda.current_stream()
    side = (stream, [torch.cuda.Stream(device=DEV) for _ in range(nbt)])
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    torch.cuda.synchronize()
    bench.launch_pipelined(pd, Xd, Yd, bufs, stream, side, steps, fused, K, evs, after_bt)
    torch.cuda.synchronize()
    for s, (t, p, pl) in enumerate(outs):
        assert int(pl.item()) == L, s
        assert float(t.item()) == ref_total, s
        assert np.array_equal(p[:L].cpu().numpy(), ref_path), s
