"""Thin Python binding of libpardtw.so (declared in include/pardtw.h).

Argument marshalling only: every step of the alignment runs in the library's
HIP kernels. PyTorch supplies device memory and the current stream. The
library must have been built (``python -m paper_2607_15478_amd.build``);
importing this module without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpardtw.so")

PARDTW_OK = 0
PAIR_OK = 0
PAIR_INFEASIBLE = 1
PREC_F32 = 0
PREC_BF16 = 1
LAYOUT_ROW = 0
LAYOUT_PANEL = 1
LAYOUT_PANEL_BAND = 2  # panel layout, only the 8-row groups the DP reads (the path band) are written
LAYOUT_PANEL_SUBSEQ_BAND = 3  # panel layout, only the groups the subsequence DP reads are written
NSDTW = 0
WSDTW = 1
PLAN_FUSED_COST = 1  # plans whose DP computes the costs itself (FP32, d <= 16)
NOALLOC_SCRATCH_BYTES = 64 << 20  # static device workspace of pardtw_dp_noalloc

STATUS_NAMES = {0: "OK", 1: "ERR_INVALID_ARG", 2: "ERR_WORKSPACE", 3: "ERR_HIP", 4: "ERR_UNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2607_15478_amd.build` first")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t
_E = ctypes.c_int


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_lib_cost_elems = _sig("pardtw_cost_elems", _SZ, [_I64, _I64, _E])
_lib_bp_bytes = _sig("pardtw_bp_bytes", _SZ, [_I64, _I64])
_lib_band = _sig("pardtw_band_groups", _E, [_I64, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64)])
_lib_dp_ws = _sig("pardtw_dp_workspace_bytes", _SZ, [_I64, _I64])
_lib_cost = _sig("pardtw_cost", _E, [_P, _P, _I64, _I64, _I64, _E, _E, _P, _P])
_lib_dp = _sig("pardtw_dp", _E, [_P, _E, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_dp_noalloc = _sig("pardtw_dp_noalloc", _E, [_P, _E, _I64, _I64, _P, _P, _P, _P])
_lib_dp_ex = _sig("pardtw_dp_ex", _E, [_P, _E, _I64, _I64, _P, _P, _P, _P, _SZ, _I32, _P])
_lib_bt = _sig("pardtw_backtrace", _E, [_P, _I64, _I64, _P, _P, _P, _P])
_lib_dp_fused = _sig("pardtw_dp_fused", _E, [_P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _SZ, _I32, _P])
_lib_sub_dp_fused = _sig("pardtw_subseq_dp_fused", _E, [_P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_unpack = _sig("pardtw_bp_unpack", _E, [_P, _I64, _I64, _P, _P])
_lib_bp2_bytes = _sig("pardtw_bp2_bytes", _SZ, [_I64, _I64])
_lib_dp_packed = _sig("pardtw_dp_packed", _E, [_P, _E, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_dp_fused_packed = _sig("pardtw_dp_fused_packed", _E, [_P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_bt_packed = _sig("pardtw_backtrace_packed", _E, [_P, _I64, _I64, _P, _P, _P, _P])
_lib_unpack2 = _sig("pardtw_bp2_unpack", _E, [_P, _I64, _I64, _P, _P])
_lib_bt_par_bytes = _sig("pardtw_backtrace_parallel_bytes", _SZ, [_I64, _I64])
_lib_bt_par = _sig("pardtw_backtrace_parallel", _E, [_P, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_bt_packed_par = _sig("pardtw_backtrace_packed_parallel", _E, [_P, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_ckpt_bytes = _sig("pardtw_ckpt_bytes", _SZ, [_I64, _I64, _I32])
_lib_dp_ckpt = _sig("pardtw_dp_fused_ckpt", _E, [_P, _P, _I64, _I64, _I64, _I32, _P, _SZ, _P, _P, _P, _SZ, _P])
_lib_ckpt_bt = _sig("pardtw_ckpt_backtrace", _E, [_P, _P, _I64, _I64, _I64, _I32, _P, _SZ, _P, _P, _P, _P])
_lib_ckpt_bt_par_bytes = _sig("pardtw_ckpt_backtrace_parallel_bytes", _SZ, [_I64, _I64, _I32])
_lib_ckpt_bt_par = _sig("pardtw_ckpt_backtrace_parallel", _E,
                        [_P, _P, _I64, _I64, _I64, _I32, _P, _SZ, _P, _P, _P, _P, _SZ, _P])
_lib_total = _sig("pardtw_path_total", _E, [_P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_total_bytes = _sig("pardtw_path_total_bytes", _SZ, [])
_lib_grad = _sig("pardtw_path_grad", _E, [_P, _P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P])
_lib_plan_create = _sig("pardtw_plan_create_ex", _E, [_I32, _P, _P, _I64, _E, _I32, ctypes.POINTER(_P)])
_lib_plan_ws = _sig("pardtw_plan_workspace_bytes", _SZ, [_P])
_lib_plan_cap = _sig("pardtw_plan_path_capacity", _I64, [_P])
_lib_plan_destroy = _sig("pardtw_plan_destroy", None, [_P])
_lib_align_batch = _sig("pardtw_align_batch", _E, [_P, _P, _P, _P, _SZ, _P, _P, _P, _P, _P])
_lib_grad_batch = _sig("pardtw_path_grad_batch", _E, [_P, _P, _P, _P, _P, _P, _P, _P, _P])
_lib_plan_nsched = _sig("pardtw_plan_num_schedules", _I32, [_P])
_lib_plan_sched = _sig("pardtw_plan_schedule", _E, [_P, _I32, _P, _P, _P])
_lib_plan_selected = _sig("pardtw_plan_selected", _I32, [_P])
_lib_plan_select = _sig("pardtw_plan_select", _E, [_P, _I32])
_lib_plan_autotune = _sig("pardtw_plan_autotune", _E, [_P, _P, _P, _P, _SZ, _P, _P, _P, _P, _I32, _P, _P])
_lib_status_string = _sig("pardtw_status_string", ctypes.c_char_p, [_E])
_lib_sub_band = _sig("pardtw_subseq_band_groups", _E, [_I64, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64)])
_lib_sub_dp = _sig("pardtw_subseq_dp", _E, [_P, _E, _I64, _I64, _P, _P, _P, _P, _SZ, _P])
_lib_sub_bt = _sig("pardtw_subseq_backtrace", _E, [_P, _I64, _I64, _P, _P, _P, _P])
_lib_seg_ws = _sig("pardtw_segment_workspace_bytes", _SZ, [_I64, _I64])
_lib_seg_ends = _sig("pardtw_segment_ends", _E, [_P, _I64, _I64, _I64, _I32, _P, _SZ, _P, _P, _P, _P])
_lib_segplan_create = _sig("pardtw_segplan_create", _E, [_I64, _I64, _I32, _I64, _E, _I32, _I32,
                                                         ctypes.POINTER(_P)])
_lib_segplan_scores = _sig("pardtw_segplan_scores_offset", _I64, [_P])
_lib_segplan_hop = _sig("pardtw_segplan_hop", _I64, [_P])
_lib_segplan_fstart = _sig("pardtw_segplan_fragment_start", _I64, [_P, ctypes.c_int32])
_lib_seg_align = _sig("pardtw_segmental_align", _E, [_P, _P, _P, _P, _SZ, _P, _P, _P, _P, _P, _P])
_lib_segplan_autotune = _sig("pardtw_segplan_autotune", _E, [_P, _P, _P, _P, _SZ, _I32, _P, _P])


class PardtwError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != PARDTW_OK:
        msg = _lib_status_string(rc).decode()
        raise PardtwError(f"{what}: {STATUS_NAMES.get(rc, rc)} ({msg})")


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


# ---- sizes ------------------------------------------------------------------
def pardtw_cost_elems(n: int, m: int, layout: int = LAYOUT_PANEL) -> int:
    return int(_lib_cost_elems(n, m, layout))


def pardtw_band_groups(n: int, m: int, p: int):
    """(lo, hi): the 8-row groups of panel p in the path band (empty if lo > hi)."""
    lo, hi = _I64(), _I64()
    _check(_lib_band(n, m, p, ctypes.byref(lo), ctypes.byref(hi)), "pardtw_band_groups")
    return lo.value, hi.value


def pardtw_bp_bytes(n: int, m: int) -> int:
    return int(_lib_bp_bytes(n, m))


def pardtw_dp_workspace_bytes(n: int, m: int) -> int:
    return int(_lib_dp_ws(n, m))


# ---- the four steps of the hot path -----------------------------------------
def pardtw_cost(X: torch.Tensor, Y: torch.Tensor, C: torch.Tensor, prec: int = PREC_F32,
                layout: int = LAYOUT_PANEL, stream=None) -> torch.Tensor:
    _dev_f32(X, "X"), _dev_f32(Y, "Y"), _dev_f32(C, "C")
    n, d = X.shape
    m, d2 = Y.shape
    if d2 != d:
        raise ValueError("X and Y feature dimensions differ")
    if C.numel() < pardtw_cost_elems(n, m, layout):
        raise ValueError("C is too small for this layout")
    _check(_lib_cost(_ptr(X), _ptr(Y), n, m, d, prec, layout, _ptr(C), _stream(stream)), "pardtw_cost")
    return C


def pardtw_dp(C: torch.Tensor, n: int, m: int, bp: torch.Tensor, total: torch.Tensor, status: torch.Tensor,
              workspace: torch.Tensor, layout: int = LAYOUT_PANEL, stream=None, panels_per_workgroup=None):
    _dev_f32(C, "C")
    if C.numel() < pardtw_cost_elems(n, m, layout):
        raise ValueError("C is too small for this layout")
    if bp.dtype != torch.uint8 or bp.numel() < pardtw_bp_bytes(n, m):
        raise ValueError("bp must be a uint8 tensor of pardtw_bp_bytes(n, m) bytes")
    if total.dtype != torch.float32 or status.dtype != torch.int32:
        raise ValueError("total must be float32 and status int32")
    ws_bytes = workspace.numel() * workspace.element_size()
    if panels_per_workgroup is None:
        _check(_lib_dp(_ptr(C), layout, n, m, _ptr(bp), _ptr(total), _ptr(status), _ptr(workspace), ws_bytes,
                       _stream(stream)), "pardtw_dp")
    else:
        _check(_lib_dp_ex(_ptr(C), layout, n, m, _ptr(bp), _ptr(total), _ptr(status), _ptr(workspace), ws_bytes,
                          int(panels_per_workgroup), _stream(stream)), "pardtw_dp_ex")


def pardtw_dp_noalloc(C: torch.Tensor, n: int, m: int, bp: torch.Tensor, total: torch.Tensor, status: torch.Tensor,
                      layout: int = LAYOUT_PANEL, stream=None):
    """pardtw_dp without a workspace argument: the library's static device
    scratch serves as workspace (sizes up to NOALLOC_SCRATCH_BYTES of it)."""
    _dev_f32(C, "C")
    if C.numel() < pardtw_cost_elems(n, m, layout):
        raise ValueError("C is too small for this layout")
    if bp.dtype != torch.uint8 or bp.numel() < pardtw_bp_bytes(n, m):
        raise ValueError("bp must be a uint8 tensor of pardtw_bp_bytes(n, m) bytes")
    if total.dtype != torch.float32 or status.dtype != torch.int32:
        raise ValueError("total must be float32 and status int32")
    _check(_lib_dp_noalloc(_ptr(C), layout, n, m, _ptr(bp), _ptr(total), _ptr(status), _stream(stream)),
           "pardtw_dp_noalloc")


def pardtw_path_total_bytes() -> int:
    return int(_lib_total_bytes())


def pardtw_path_total(X: torch.Tensor, Y: torch.Tensor, path: torch.Tensor, path_len: torch.Tensor,
                      total: torch.Tensor, workspace: Optional[torch.Tensor] = None, stream=None):
    """The path's cost summed in two-float arithmetic (compensated total).
    Without `workspace` one of pardtw_path_total_bytes() is allocated."""
    _dev_f32(X, "X"), _dev_f32(Y, "Y"), _dev_f32(total, "total")
    if path.dtype != torch.int32 or path_len.dtype != torch.int32:
        raise ValueError("path and path_len must be int32")
    n, d = X.shape
    m = Y.shape[0]
    if workspace is None:
        workspace = torch.empty(pardtw_path_total_bytes(), dtype=torch.uint8, device=X.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_total(_ptr(X), _ptr(Y), n, m, d, _ptr(path), _ptr(path_len), _ptr(total), _ptr(workspace),
                      ws_bytes, _stream(stream)), "pardtw_path_total")


def pardtw_dp_fused(X: torch.Tensor, Y: torch.Tensor, bp: torch.Tensor, total: torch.Tensor, status: torch.Tensor,
                    workspace: torch.Tensor, stream=None, panels_per_workgroup: int = 0):
    """The DP with the cost computed inside it (FP32 features, d <= 16)."""
    _dev_f32(X, "X"), _dev_f32(Y, "Y")
    n, d = X.shape
    m = Y.shape[0]
    if bp.dtype != torch.uint8 or bp.numel() < pardtw_bp_bytes(n, m):
        raise ValueError("bp must be a uint8 tensor of pardtw_bp_bytes(n, m) bytes")
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_dp_fused(_ptr(X), _ptr(Y), n, m, d, _ptr(bp), _ptr(total), _ptr(status), _ptr(workspace), ws_bytes,
                         int(panels_per_workgroup), _stream(stream)), "pardtw_dp_fused")


CKPT_MAX_ROWS = 256  # the largest block of rows the checkpointed backtrace's window holds


def pardtw_ckpt_bytes(n: int, m: int, rows_per_block: int) -> int:
    """Bytes of the checkpoint rows for blocks of `rows_per_block` rows (0 on bad args)."""
    return int(_lib_ckpt_bytes(n, m, rows_per_block))


def pardtw_dp_fused_ckpt(X: torch.Tensor, Y: torch.Tensor, rows_per_block: int, ckpt: torch.Tensor,
                         total: torch.Tensor, status: torch.Tensor, workspace: torch.Tensor, stream=None):
    """The fused DP writing no codes, only the D rows every block of rows starts from."""
    _dev_f32(X, "X"), _dev_f32(Y, "Y")
    n, d = X.shape
    m = Y.shape[0]
    ws_bytes = workspace.numel() * workspace.element_size()
    ck_bytes = ckpt.numel() * ckpt.element_size()
    _check(_lib_dp_ckpt(_ptr(X), _ptr(Y), n, m, d, int(rows_per_block), _ptr(ckpt) if ck_bytes else None, ck_bytes,
                        _ptr(total), _ptr(status), _ptr(workspace), ws_bytes, _stream(stream)),
           "pardtw_dp_fused_ckpt")


def pardtw_ckpt_backtrace(X: torch.Tensor, Y: torch.Tensor, rows_per_block: int, ckpt: torch.Tensor,
                          status: torch.Tensor, path: torch.Tensor, path_len: torch.Tensor, stream=None):
    """The path from the checkpoints of pardtw_dp_fused_ckpt (same X, Y and rows_per_block)."""
    _dev_f32(X, "X"), _dev_f32(Y, "Y")
    n, d = X.shape
    m = Y.shape[0]
    if path.dtype != torch.int32 or path.numel() < 2 * min(n, m):
        raise ValueError("path must be int32 with room for 2*min(n, m) entries")
    ck_bytes = ckpt.numel() * ckpt.element_size()
    _check(_lib_ckpt_bt(_ptr(X), _ptr(Y), n, m, d, int(rows_per_block), _ptr(ckpt) if ck_bytes else None, ck_bytes,
                        _ptr(status), _ptr(path), _ptr(path_len), _stream(stream)), "pardtw_ckpt_backtrace")


def pardtw_ckpt_backtrace_parallel_bytes(n: int, m: int, rows_per_block: int) -> int:
    return int(_lib_ckpt_bt_par_bytes(n, m, int(rows_per_block)))


def pardtw_ckpt_backtrace_parallel(X: torch.Tensor, Y: torch.Tensor, rows_per_block: int, ckpt: torch.Tensor,
                                   status: torch.Tensor, path: torch.Tensor, path_len: torch.Tensor,
                                   workspace: torch.Tensor, stream=None):
    """pardtw_ckpt_backtrace's path, split into runs of blocks walked at once
    (workspace: pardtw_ckpt_backtrace_parallel_bytes(n, m, rows_per_block) bytes)."""
    _dev_f32(X, "X"), _dev_f32(Y, "Y")
    n, d = X.shape
    m = Y.shape[0]
    if path.dtype != torch.int32 or path.numel() < 2 * min(n, m):
        raise ValueError("path must be int32 with room for 2*min(n, m) entries")
    ck_bytes = ckpt.numel() * ckpt.element_size()
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_ckpt_bt_par(_ptr(X), _ptr(Y), n, m, d, int(rows_per_block), _ptr(ckpt) if ck_bytes else None,
                            ck_bytes, _ptr(status), _ptr(path), _ptr(path_len), _ptr(workspace), ws_bytes,
                            _stream(stream)), "pardtw_ckpt_backtrace_parallel")


def pardtw_backtrace(bp: torch.Tensor, n: int, m: int, status: torch.Tensor, path: torch.Tensor,
                     path_len: torch.Tensor, stream=None):
    if path.dtype != torch.int32 or path.numel() < 2 * min(n, m):
        raise ValueError("path must be int32 with room for 2*min(n, m) entries")
    _check(_lib_bt(_ptr(bp), n, m, _ptr(status), _ptr(path), _ptr(path_len), _stream(stream)),
           "pardtw_backtrace")


def pardtw_bp2_bytes(n: int, m: int) -> int:
    return int(_lib_bp2_bytes(n, m))


def _check_bp2(bp2: torch.Tensor, n: int, m: int):
    if bp2.dtype != torch.uint8 or bp2.numel() < pardtw_bp2_bytes(n, m) or bp2.data_ptr() % 16:
        raise ValueError("bp2 must be a 16-byte aligned uint8 tensor of pardtw_bp2_bytes(n, m) bytes")


def pardtw_dp_packed(C: torch.Tensor, n: int, m: int, bp2: torch.Tensor, total: torch.Tensor,
                     status: torch.Tensor, workspace: torch.Tensor, layout: int = LAYOUT_PANEL_BAND, stream=None):
    """pardtw_dp with 2-bit packed codes."""
    _dev_f32(C, "C")
    if C.numel() < pardtw_cost_elems(n, m, layout):
        raise ValueError("C is too small for this layout")
    _check_bp2(bp2, n, m)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_dp_packed(_ptr(C), layout, n, m, _ptr(bp2), _ptr(total), _ptr(status), _ptr(workspace), ws_bytes,
                          _stream(stream)), "pardtw_dp_packed")


def pardtw_dp_fused_packed(X: torch.Tensor, Y: torch.Tensor, bp2: torch.Tensor, total: torch.Tensor,
                           status: torch.Tensor, workspace: torch.Tensor, stream=None):
    """pardtw_dp_fused with 2-bit packed codes."""
    _dev_f32(X, "X"), _dev_f32(Y, "Y")
    n, d = X.shape
    m = Y.shape[0]
    _check_bp2(bp2, n, m)
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_dp_fused_packed(_ptr(X), _ptr(Y), n, m, d, _ptr(bp2), _ptr(total), _ptr(status), _ptr(workspace),
                                ws_bytes, _stream(stream)), "pardtw_dp_fused_packed")


def pardtw_backtrace_packed(bp2: torch.Tensor, n: int, m: int, status: torch.Tensor, path: torch.Tensor,
                            path_len: torch.Tensor, stream=None):
    _check_bp2(bp2, n, m)
    if path.dtype != torch.int32 or path.numel() < 2 * min(n, m):
        raise ValueError("path must be int32 with room for 2*min(n, m) entries")
    _check(_lib_bt_packed(_ptr(bp2), n, m, _ptr(status), _ptr(path), _ptr(path_len), _stream(stream)),
           "pardtw_backtrace_packed")


def pardtw_backtrace_parallel_bytes(n: int, m: int) -> int:
    return int(_lib_bt_par_bytes(n, m))


def pardtw_backtrace_parallel(bp: torch.Tensor, n: int, m: int, status: torch.Tensor, path: torch.Tensor,
                              path_len: torch.Tensor, workspace: torch.Tensor, stream=None, packed: bool = False):
    """The split walk (the same path as pardtw_backtrace / pardtw_backtrace_packed);
    `workspace` holds pardtw_backtrace_parallel_bytes(n, m) bytes, 16-byte aligned."""
    if packed:
        _check_bp2(bp, n, m)
    if path.dtype != torch.int32 or path.numel() < 2 * min(n, m):
        raise ValueError("path must be int32 with room for 2*min(n, m) entries")
    ws_bytes = workspace.numel() * workspace.element_size()
    fn, name = (_lib_bt_packed_par, "pardtw_backtrace_packed_parallel") if packed else \
        (_lib_bt_par, "pardtw_backtrace_parallel")
    _check(fn(_ptr(bp), n, m, _ptr(status), _ptr(path), _ptr(path_len), _ptr(workspace), ws_bytes,
              _stream(stream)), name)


def pardtw_bp2_unpack(bp2: torch.Tensor, n: int, m: int, out: Optional[torch.Tensor] = None, stream=None):
    if out is None:
        out = torch.empty((n, m), dtype=torch.int8, device=bp2.device)
    _check(_lib_unpack2(_ptr(bp2), n, m, _ptr(out), _stream(stream)), "pardtw_bp2_unpack")
    return out


def pardtw_bp_unpack(bp: torch.Tensor, n: int, m: int, out: Optional[torch.Tensor] = None, stream=None):
    if out is None:
        out = torch.empty((n, m), dtype=torch.int8, device=bp.device)
    _check(_lib_unpack(_ptr(bp), n, m, _ptr(out), _stream(stream)), "pardtw_bp_unpack")
    return out


def pardtw_path_grad(X, Y, path, path_len, g_total, dX, dY, stream=None):
    n, d = X.shape
    m = Y.shape[0]
    _check(_lib_grad(_ptr(X), _ptr(Y), n, m, d, _ptr(path), _ptr(path_len), _ptr(g_total), _ptr(dX), _ptr(dY),
                     _stream(stream)), "pardtw_path_grad")


# ---- convenience: buffers + the whole path for one pair ---------------------
class Workspace:
    """Device buffers for one (n, m) alignment, reusable across calls."""

    def __init__(self, n: int, m: int, device="cuda", layout: int = LAYOUT_PANEL_BAND, cost: bool = True,
                 ckpt_rows: int = 0, packed: bool = False):
        self.n, self.m, self.layout = n, m, layout
        # no cost buffer when the DP computes the costs itself; with ckpt_rows
        # (checkpointed backtrace, fused cost) no codes either
        self.ckpt_rows = int(ckpt_rows)
        if self.ckpt_rows and cost:
            raise ValueError("the checkpointed DP computes its costs itself (cost=False)")
        self.C = torch.empty(pardtw_cost_elems(n, m, layout) if cost else 0, dtype=torch.float32, device=device)
        # packed: codes 2 bits per cell (pardtw_dp_packed / pardtw_dp_fused_packed)
        self.packed = bool(packed)
        code_bytes = pardtw_bp2_bytes(n, m) if self.packed else pardtw_bp_bytes(n, m)
        self.bp = torch.empty(0 if self.ckpt_rows else code_bytes, dtype=torch.uint8, device=device)
        if self.ckpt_rows and (self.ckpt_rows % 16 or not 16 <= self.ckpt_rows <= CKPT_MAX_ROWS):
            raise ValueError(f"ckpt_rows must be a multiple of 16 in [16, {CKPT_MAX_ROWS}]")
        ck_bytes = pardtw_ckpt_bytes(n, m, self.ckpt_rows) if self.ckpt_rows else 0
        self.ckpt = torch.empty(ck_bytes // 4, dtype=torch.float32, device=device)
        self.ws = torch.zeros(pardtw_dp_workspace_bytes(n, m), dtype=torch.uint8, device=device)
        self.total = torch.empty(1, dtype=torch.float32, device=device)
        self.total_comp = torch.empty(1, dtype=torch.float32, device=device)  # pardtw_path_total's output
        self.total_ws = torch.empty(pardtw_path_total_bytes(), dtype=torch.uint8, device=device)
        self.status = torch.empty(1, dtype=torch.int32, device=device)
        self.path = torch.empty((min(n, m), 2), dtype=torch.int32, device=device)
        self.path_len = torch.empty(1, dtype=torch.int32, device=device)
        # the split backtrace's segments (8 B per row; with checkpoints, runs of blocks)
        self.bt_ws = torch.empty(pardtw_ckpt_backtrace_parallel_bytes(n, m, self.ckpt_rows) if self.ckpt_rows
                                 else pardtw_backtrace_parallel_bytes(n, m), dtype=torch.uint8, device=device)


def align_into(X: torch.Tensor, Y: torch.Tensor, w: Workspace, prec: int = PREC_F32, stream=None,
               fused: bool = False, serial_backtrace: bool = False):
    """cost -> dp -> backtrace on the given stream, results left in w (with
    `fused`, the DP computes the costs itself and w.C is not used). The
    backtrace is the split walk unless `serial_backtrace` (same path)."""
    n, m = X.shape[0], Y.shape[0]
    if w.ckpt_rows:
        if prec != PREC_F32:
            raise ValueError("the checkpointed DP computes FP32 costs")
        pardtw_dp_fused_ckpt(X, Y, w.ckpt_rows, w.ckpt, w.total, w.status, w.ws, stream)
        if serial_backtrace:
            pardtw_ckpt_backtrace(X, Y, w.ckpt_rows, w.ckpt, w.status, w.path, w.path_len, stream)
        else:
            pardtw_ckpt_backtrace_parallel(X, Y, w.ckpt_rows, w.ckpt, w.status, w.path, w.path_len, w.bt_ws, stream)
        return w
    if fused:
        if prec != PREC_F32:
            raise ValueError("the fused DP computes FP32 costs")
        if w.packed:
            pardtw_dp_fused_packed(X, Y, w.bp, w.total, w.status, w.ws, stream)
        else:
            pardtw_dp_fused(X, Y, w.bp, w.total, w.status, w.ws, stream)
    else:
        pardtw_cost(X, Y, w.C, prec, w.layout, stream)
        if w.packed:
            pardtw_dp_packed(w.C, n, m, w.bp, w.total, w.status, w.ws, w.layout, stream)
        else:
            pardtw_dp(w.C, n, m, w.bp, w.total, w.status, w.ws, w.layout, stream)
    if not serial_backtrace:
        pardtw_backtrace_parallel(w.bp, n, m, w.status, w.path, w.path_len, w.bt_ws, stream, packed=w.packed)
    elif w.packed:
        pardtw_backtrace_packed(w.bp, n, m, w.status, w.path, w.path_len, stream)
    else:
        pardtw_backtrace(w.bp, n, m, w.status, w.path, w.path_len, stream)
    return w


def align(X: torch.Tensor, Y: torch.Tensor, prec: int = PREC_F32, layout: int = LAYOUT_PANEL_BAND):
    """Exact DTW of two feature sequences on the GPU: (total, path (L,2) int32, status)."""
    w = Workspace(X.shape[0], Y.shape[0], X.device, layout)
    align_into(X, Y, w, prec)
    L = int(w.path_len.item())
    return float(w.total.item()), w.path[:L].clone(), int(w.status.item())


# ---- batched form -----------------------------------------------------------
class Plan:
    """A batch of pairs with fixed lengths (pardtw_plan_create). Buffers are
    packed as the C header describes; `buffers()` allocates a matching set."""

    def __init__(self, ns, ms, d: int, prec: int = PREC_F32, fused: bool = False):
        ns = [int(v) for v in ns]
        ms = [int(v) for v in ms]
        if len(ns) != len(ms) or not ns:
            raise ValueError("ns and ms must be non-empty and of equal length")
        self.ns, self.ms, self.d, self.prec = ns, ms, int(d), prec
        self.batch = len(ns)
        n_arr = (ctypes.c_int64 * self.batch)(*ns)
        m_arr = (ctypes.c_int64 * self.batch)(*ms)
        h = _P()
        self.fused = bool(fused)
        _check(_lib_plan_create(self.batch, n_arr, m_arr, self.d, prec, PLAN_FUSED_COST if fused else 0,
                                ctypes.byref(h)), "pardtw_plan_create_ex")
        self._h = h
        self.workspace_bytes = int(_lib_plan_ws(h))
        self.path_capacity = int(_lib_plan_cap(h))
        self.x_off = [0] * self.batch
        self.y_off = [0] * self.batch
        self.p_off = [0] * self.batch
        xo = yo = po = 0
        for b in range(self.batch):
            self.x_off[b], self.y_off[b], self.p_off[b] = xo, yo, po
            xo += ns[b]
            yo += ms[b]
            po += min(ns[b], ms[b])

    def __del__(self, _destroy=_lib_plan_destroy):
        # the destroy call is bound here: at interpreter exit the module's
        # globals may already be gone when the last plan is collected
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
            self._h = None

    def buffers(self, device="cuda"):
        """Output and workspace tensors for this plan (workspace zeroed)."""
        return dict(
            workspace=torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=device),
            totals=torch.empty(self.batch, dtype=torch.float32, device=device),
            paths=torch.empty((self.path_capacity, 2), dtype=torch.int32, device=device),
            path_len=torch.empty(self.batch, dtype=torch.int32, device=device),
            status=torch.empty(self.batch, dtype=torch.int32, device=device),
        )

    def _args(self, Xp, Yp, buf):
        _dev_f32(Xp, "X_packed"), _dev_f32(Yp, "Y_packed")
        if Xp.shape != (sum(self.ns), self.d) or Yp.shape != (sum(self.ms), self.d):
            raise ValueError("packed features do not match the plan")
        ws = buf["workspace"]
        return (_ptr(Xp), _ptr(Yp), _ptr(ws), ws.numel() * ws.element_size(), _ptr(buf["totals"]),
                _ptr(buf["paths"]), _ptr(buf["path_len"]), _ptr(buf["status"]))

    def align(self, Xp: torch.Tensor, Yp: torch.Tensor, buf: dict, stream=None):
        _check(_lib_align_batch(self._h, *self._args(Xp, Yp, buf), _stream(stream)), "pardtw_align_batch")

    def autotune(self, Xp: torch.Tensor, Yp: torch.Tensor, buf: dict, reps: int = 2, stream=None) -> float:
        best = ctypes.c_float(0.0)
        _check(_lib_plan_autotune(self._h, *self._args(Xp, Yp, buf), int(reps), ctypes.byref(best),
                                  _stream(stream)), "pardtw_plan_autotune")
        return float(best.value)

    @property
    def num_schedules(self) -> int:
        return int(_lib_plan_nsched(self._h))

    def schedule(self, index: int = -1):
        nw, order, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib_plan_sched(self._h, int(index), ctypes.byref(nw), ctypes.byref(order), ctypes.byref(wg)),
               "pardtw_plan_schedule")
        return dict(panels_per_workgroup=nw.value, order=("breadth", "depth")[order.value], workgroups=wg.value)

    @property
    def selected(self) -> int:
        return int(_lib_plan_selected(self._h))

    def select(self, index: int):
        _check(_lib_plan_select(self._h, int(index)), "pardtw_plan_select")

    def path(self, buf: dict, b: int) -> torch.Tensor:
        L = int(buf["path_len"][b].item())
        return buf["paths"][self.p_off[b]: self.p_off[b] + L]

    def path_grad(self, Xp, Yp, buf, g_totals, dXp, dYp, stream=None):
        _check(_lib_grad_batch(self._h, _ptr(Xp), _ptr(Yp), _ptr(buf["paths"]), _ptr(buf["path_len"]),
                               _ptr(g_totals), _ptr(dXp), _ptr(dYp), _stream(stream)), "pardtw_path_grad_batch")


def pack(pairs, device="cuda"):
    """[(X_b, Y_b)] numpy pairs -> (X_packed, Y_packed) device tensors."""
    import numpy as np
    Xp = torch.from_numpy(np.ascontiguousarray(np.concatenate([p[0] for p in pairs]), dtype=np.float32)).to(device)
    Yp = torch.from_numpy(np.ascontiguousarray(np.concatenate([p[1] for p in pairs]), dtype=np.float32)).to(device)
    return Xp, Yp


# ---- subsequence DTW and Segmental DTW --------------------------------------
def pardtw_subseq_band_groups(n: int, m: int, p: int):
    """(lo, hi): the 8-row groups of panel p in the subsequence band."""
    lo, hi = _I64(), _I64()
    _check(_lib_sub_band(n, m, p, ctypes.byref(lo), ctypes.byref(hi)), "pardtw_subseq_band_groups")
    return lo.value, hi.value


def pardtw_subseq_dp(C: torch.Tensor, n: int, m: int, bp: torch.Tensor, scores: torch.Tensor, status: torch.Tensor,
                     workspace: torch.Tensor, layout: int = LAYOUT_PANEL, stream=None):
    _dev_f32(C, "C"), _dev_f32(scores, "scores")
    if C.numel() < pardtw_cost_elems(n, m, layout):
        raise ValueError("C is too small for this layout")
    if bp.dtype != torch.uint8 or bp.numel() < pardtw_bp_bytes(n, m):
        raise ValueError("bp must be a uint8 tensor of pardtw_bp_bytes(n, m) bytes")
    if scores.numel() < m or status.dtype != torch.int32:
        raise ValueError("scores must hold m floats and status be int32")
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_sub_dp(_ptr(C), layout, n, m, _ptr(bp), _ptr(scores), _ptr(status), _ptr(workspace), ws_bytes,
                       _stream(stream)), "pardtw_subseq_dp")


def pardtw_subseq_dp_fused(X: torch.Tensor, Y: torch.Tensor, bp: torch.Tensor, scores: torch.Tensor,
                           status: torch.Tensor, workspace: torch.Tensor, stream=None):
    _dev_f32(X, "X"), _dev_f32(Y, "Y"), _dev_f32(scores, "scores")
    n, d = X.shape
    m = Y.shape[0]
    if bp.dtype != torch.uint8 or bp.numel() < pardtw_bp_bytes(n, m) or scores.numel() < m:
        raise ValueError("bp must hold pardtw_bp_bytes(n, m) bytes and scores m floats")
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_sub_dp_fused(_ptr(X), _ptr(Y), n, m, d, _ptr(bp), _ptr(scores), _ptr(status), _ptr(workspace),
                             ws_bytes, _stream(stream)), "pardtw_subseq_dp_fused")


def pardtw_subseq_backtrace(bp: torch.Tensor, n: int, m: int, end_col: torch.Tensor, path: torch.Tensor,
                            path_len: torch.Tensor, stream=None):
    if path.dtype != torch.int32 or path.numel() < 2 * n:
        raise ValueError("path must be int32 with room for 2*n entries")
    if end_col.dtype != torch.int32:
        raise ValueError("end_col must be int32")
    _check(_lib_sub_bt(_ptr(bp), n, m, _ptr(end_col), _ptr(path), _ptr(path_len), _stream(stream)),
           "pardtw_subseq_backtrace")


def pardtw_segment_workspace_bytes(nfrag: int, m: int) -> int:
    return int(_lib_seg_ws(nfrag, m))


def pardtw_segment_ends(scores: torch.Tensor, nfrag: int, m: int, hop: int, variant: int, workspace: torch.Tensor,
                        ends: torch.Tensor, total: torch.Tensor, status: torch.Tensor, stream=None):
    _dev_f32(scores, "scores")
    if scores.numel() < nfrag * m or ends.dtype != torch.int32 or ends.numel() < nfrag:
        raise ValueError("scores must hold nfrag*m floats and ends nfrag int32")
    ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib_seg_ends(_ptr(scores), nfrag, m, int(hop), int(variant), _ptr(workspace), ws_bytes, _ptr(ends),
                         _ptr(total), _ptr(status), _stream(stream)), "pardtw_segment_ends")


class SegPlan:
    """Segmental DTW of A (la x d) against B (lb x d) with nfrag fragments
    (pardtw_segplan_create); `buffers()` allocates the outputs and workspace."""

    def __init__(self, la: int, lb: int, nfrag: int, d: int, prec: int = PREC_F32, variant: int = WSDTW,
                 fused: bool = False):
        self.la, self.lb, self.nfrag, self.d, self.prec, self.variant = int(la), int(lb), int(nfrag), int(d), prec, variant
        self.fused = bool(fused)
        h = _P()
        _check(_lib_segplan_create(self.la, self.lb, self.nfrag, self.d, prec, int(variant),
                                   PLAN_FUSED_COST if fused else 0, ctypes.byref(h)), "pardtw_segplan_create")
        self._h = h
        self.workspace_bytes = int(_lib_plan_ws(h))
        self.scores_offset = int(_lib_segplan_scores(h))
        # the plan's own fragment split and segment hop, as the library uses them
        self.starts = [int(_lib_segplan_fstart(h, f)) for f in range(self.nfrag + 1)]
        self.hop = int(_lib_segplan_hop(h))

    def __del__(self, _destroy=_lib_plan_destroy):
        # the destroy call is bound here: at interpreter exit the module's
        # globals may already be gone when the last plan is collected
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
            self._h = None

    def buffers(self, device="cuda"):
        return dict(
            workspace=torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=device),
            total=torch.empty(1, dtype=torch.float32, device=device),
            ends=torch.empty(self.nfrag, dtype=torch.int32, device=device),
            path=torch.empty((self.la, 2), dtype=torch.int32, device=device),
            path_len=torch.empty(1, dtype=torch.int32, device=device),
            status=torch.empty(1, dtype=torch.int32, device=device),
        )

    def _check_inputs(self, A, B):
        _dev_f32(A, "A"), _dev_f32(B, "B")
        if A.shape != (self.la, self.d) or B.shape != (self.lb, self.d):
            raise ValueError("A and B do not match the plan")

    def align(self, A: torch.Tensor, B: torch.Tensor, buf: dict, stream=None):
        self._check_inputs(A, B)
        ws = buf["workspace"]
        _check(_lib_seg_align(self._h, _ptr(A), _ptr(B), _ptr(ws), ws.numel() * ws.element_size(),
                              _ptr(buf["total"]), _ptr(buf["ends"]), _ptr(buf["path"]), _ptr(buf["path_len"]),
                              _ptr(buf["status"]), _stream(stream)), "pardtw_segmental_align")

    def autotune(self, A: torch.Tensor, B: torch.Tensor, buf: dict, reps: int = 2, stream=None) -> float:
        self._check_inputs(A, B)
        ws = buf["workspace"]
        best = ctypes.c_float(0.0)
        _check(_lib_segplan_autotune(self._h, _ptr(A), _ptr(B), _ptr(ws), ws.numel() * ws.element_size(), int(reps),
                                     ctypes.byref(best), _stream(stream)), "pardtw_segplan_autotune")
        return float(best.value)

    def scores(self, buf: dict) -> torch.Tensor:
        """The stacked fragment scores S (nfrag x lb) left in the workspace."""
        ws = buf["workspace"]
        n = self.nfrag * self.lb
        return ws[self.scores_offset: self.scores_offset + 4 * n].view(torch.float32).view(self.nfrag, self.lb)

    def schedule(self, index: int = -1):
        nw, order, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib_plan_sched(self._h, int(index), ctypes.byref(nw), ctypes.byref(order), ctypes.byref(wg)),
               "pardtw_plan_schedule")
        if nw.value == 0:  # one workgroup per fragment; `order` carries its waves
            return dict(panels_per_workgroup=0, order="fragment", waves=order.value, workgroups=wg.value)
        return dict(panels_per_workgroup=nw.value, order=("breadth", "depth")[order.value], workgroups=wg.value)

    def select(self, index: int):
        _check(_lib_plan_select(self._h, int(index)), "pardtw_plan_select")

    @property
    def num_schedules(self) -> int:
        return int(_lib_plan_nsched(self._h))


def segmental(A: torch.Tensor, B: torch.Tensor, nfrag: int, variant: int = WSDTW, prec: int = PREC_F32,
              fused: bool = False):
    """Segmental DTW on the GPU: (total, ends (nfrag,), path (L,2), status)."""
    plan = SegPlan(A.shape[0], B.shape[0], nfrag, A.shape[1], prec, variant, fused)
    buf = plan.buffers(A.device)
    plan.align(A, B, buf)
    L = int(buf["path_len"].item())
    return float(buf["total"].item()), buf["ends"].clone(), buf["path"][:L].clone(), int(buf["status"].item())
