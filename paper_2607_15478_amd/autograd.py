"""PyTorch autograd wrappers of the exact ParDTW cost (argument marshalling
only: forward and backward run in libpardtw's HIP kernels).

The DTW total J = sum over the optimal path of w_ij * C[i,j] is differentiated
with the optimal path held fixed (a one-sided derivative where two paths tie),
the backpropagation through the alignment path that the paper motivates in
Sec. I. The path is returned as a non-differentiable output.
"""
from __future__ import annotations

import torch

from . import pardtw as pd


class PardtwCost(torch.autograd.Function):
    """(X [n,d], Y [m,d]) -> (total [1], path [min(n,m), 2] int32 of which the
    first path_len rows are valid, path_len [1] int32, status [1] int32)."""

    @staticmethod
    def forward(ctx, X: torch.Tensor, Y: torch.Tensor, prec: int = pd.PREC_F32):
        X = X.detach().contiguous()
        Y = Y.detach().contiguous()
        w = pd.Workspace(X.shape[0], Y.shape[0], X.device)
        pd.align_into(X, Y, w, prec)
        ctx.save_for_backward(X, Y, w.path, w.path_len)
        ctx.mark_non_differentiable(w.path, w.path_len, w.status)
        return w.total.clone(), w.path, w.path_len, w.status

    @staticmethod
    def backward(ctx, g_total, g_path, g_path_len, g_status):
        X, Y, path, path_len = ctx.saved_tensors
        dX = torch.empty_like(X)
        dY = torch.empty_like(Y)
        g = g_total.reshape(1).to(torch.float32).contiguous()
        pd.pardtw_path_grad(X, Y, path, path_len, g, dX, dY)
        return dX, dY, None


def pardtw_cost(X: torch.Tensor, Y: torch.Tensor, prec: int = pd.PREC_F32):
    """Differentiable exact DTW cost of one pair: (total as a 0-d tensor, path
    (L, 2) int32). Reading the path length synchronises the stream."""
    total, path, path_len, status = PardtwCost.apply(X, Y, prec)
    return total.reshape(()), path[: int(path_len.item())]


class PardtwBatchCost(torch.autograd.Function):
    """Packed batch -> per-pair totals [B]; paths and statuses in `buf`.

    The paths are copied at forward time and the copies saved for backward:
    the plan's kernels write `buf` through raw pointers, which torch's version
    counters do not see, so a later forward on the same buffers must not
    change the paths an earlier loss differentiates along."""

    @staticmethod
    def forward(ctx, Xp: torch.Tensor, Yp: torch.Tensor, plan: pd.Plan, buf: dict):
        Xp = Xp.detach().contiguous()
        Yp = Yp.detach().contiguous()
        plan.align(Xp, Yp, buf)
        ctx.plan = plan
        ctx.save_for_backward(Xp, Yp, buf["paths"].clone(), buf["path_len"].clone())
        return buf["totals"].clone()

    @staticmethod
    def backward(ctx, g_totals):
        Xp, Yp, paths, path_len = ctx.saved_tensors
        dX = torch.empty_like(Xp)
        dY = torch.empty_like(Yp)
        ctx.plan.path_grad(Xp, Yp, {"paths": paths, "path_len": path_len},
                           g_totals.to(torch.float32).contiguous(), dX, dY)
        return dX, dY, None, None


def pardtw_batch_cost(Xp: torch.Tensor, Yp: torch.Tensor, plan: pd.Plan, buf: dict):
    return PardtwBatchCost.apply(Xp, Yp, plan, buf)
