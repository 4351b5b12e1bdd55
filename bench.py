#!/usr/bin/env python3
"""Benchmark: exact ParDTW on one MI355X, 50000 x 60000 chroma-like pair.

One step = the whole hot path for one pair with inputs resident in HBM:
  cosine-cost MFMA GEMM (panel layout, path-band groups only) -> staircase-wavefront DP -> backtrace.
Prints one JSON line with GCUPS (N*M cells / step time), pairs/s, the DP
kernel's roofline figures (algorithmic bytes / measured kernel time against
the 8 TB/s HBM peak), and the CPU baseline leg: the FP64 oracle timed on the
whole pair (about 15 s on one host core), whose result also validates the GPU
path. `--workload batch...` runs the batched form instead (see run_batch).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DP_BYTES_PER_CELL = 5  # 4 B cost read + 1 B backtrace code written
WORKLOAD = "pair_50000x60000_d12"


def band_cells(n: int, m: int) -> int:
    """Cells that can lie on a path from (0,0) to (n-1,m-1) with the steps
    (1,1), (1,2), (2,1): per row i, the columns j with ceil(i/2) <= j <= 2i
    (reachable from the origin) and m-1-2(n-1-i) <= j <= m-1-ceil((n-1-i)/2)
    (the end reachable). The DP's own work: it reads the cost and writes the
    code of these cells and of no others that matter."""
    i = np.arange(n, dtype=np.int64)
    r = n - 1 - i
    lo = np.maximum(np.maximum((i + 1) // 2, (m - 1) - 2 * r), 0)
    hi = np.minimum(np.minimum(2 * i, (m - 1) - (r + 1) // 2), m - 1)
    return int(np.maximum(hi - lo + 1, 0).sum())


def subseq_band_cells(n: int, m: int) -> int:
    """The same for subsequence DTW (free start on row 0, free end on row
    n-1): row 0 reaches (i, j) iff ceil(i/2) <= j, and (i, j) reaches row n-1
    iff j <= m-1-ceil((n-1-i)/2)."""
    i = np.arange(n, dtype=np.int64)
    lo = (i + 1) // 2
    hi = np.minimum((m - 1) - (n - i) // 2, m - 1)
    return int(np.maximum(hi - lo + 1, 0).sum())


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-validate", action="store_true", help="time the oracle but skip the path check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline leg (and validation)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "dp_traffic.json"))
    ap.add_argument("--nfrag", type=int, default=32, help="segmental workloads: fragments of sequence A")
    ap.add_argument("--fused", action="store_true",
                    help="the DP computes the costs itself (no cost matrix; FP32 d <= 16, or BF16 operands "
                         "d <= 128 for batches). Batch and segmental workloads use it by default for FP32 "
                         "d <= 16, where it is the faster form")
    ap.add_argument("--materialised", action="store_true",
                    help="batch and segmental workloads: the cost GEMM writes the cost matrix and the DP reads "
                         "it (the default for pairs)")
    ap.add_argument("--variant", choices=["wsdtw", "nsdtw"], default="wsdtw", help="segmental workloads")
    ap.add_argument("--pipelined", action="store_true",
                    help="pair workloads: run each pair's backtrace on a second stream beside the next pair's "
                         "cost and DP (the default runs each step's backtrace before the next step's cost)")
    ap.add_argument("--serial", action="store_true",
                    help="pair workloads: the serial schedule (the default; overrides --pipelined)")
    ap.add_argument("--packed", action="store_true",
                    help="pair workloads: codes packed 2 bits per cell (pardtw_dp_packed / pardtw_dp_fused_packed "
                         "and pardtw_backtrace_packed), a memory mode")
    ap.add_argument("--graph", action="store_true",
                    help="pair workloads, serial schedule: capture one step as a hipGraph and time its replays "
                         "(stage times from eager steps before the timed region)")
    ap.add_argument("--walk", choices=["auto", "split", "serial"], default="auto",
                    help="pair workloads: the backtrace, split walk (pardtw_backtrace_parallel, many workgroups) "
                         "or one-workgroup walk (pardtw_backtrace); the same path. auto: split in the serial "
                         "schedule (it shortens the step), one workgroup in the pipelined one (it hides beside "
                         "the next DP on one CU, where the split walk would take CUs from that DP)")
    ap.add_argument("--ckpt", type=int, default=0, metavar="K",
                    help="checkpointed DTW: fused DP keeping only D rows every K rows, then the recomputing "
                         "backtrace (no code matrix; K a multiple of 16 in [16, 256])")
    ap.add_argument("--no-comp-total", action="store_true",
                    help="pair workloads: skip the compensated path total (pardtw_path_total) after each backtrace")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="segmental workloads: skip the deviation from the exact DTW path")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


def host_threads() -> int:
    """Host threads for the oracle's all-core leg: the CPUs this process may
    run on, capped by OMP_NUM_THREADS when it is set."""
    n = len(os.sched_getaffinity(0))
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n, cap) if cap > 0 else n)


# Pairs above this many cells are too large for the oracle's full sweep (a
# 600000 x 600000 pair would take about half an hour on one core).
ORACLE_MAX_CELLS = 5e9
ORACLE_SAMPLE_FRAMES = 20000


def workspace_device_bytes(w) -> int:
    """Device bytes one pair's workspace holds: cost matrix, codes or
    checkpoints, DP workspace (header, boundary records, row norms), path."""
    return int(sum(t.numel() * t.element_size()
                   for t in (w.C, w.bp, w.ws, w.ckpt, w.path, w.path_len, w.total, w.status) if t is not None))


def cpu_baseline_pair(X, Y, path, total, validate=True, comp=None):
    """The oracle (single-threaded FP64 DTW with codes) timed on the whole pair;
    its result is then used to check the GPU path and total. The only use of
    the oracle in this script. A pair too large for it is timed on its
    leading 20000 x 20000 frames, and its GPU path is checked for legality
    and rescored in FP64 against the GPU total."""
    import oracle
    from tests import parity
    n, m = len(X), len(Y)
    if n * m > ORACLE_MAX_CELLS:
        s = ORACLE_SAMPLE_FRAMES
        threads = host_threads()
        t0 = time.perf_counter()
        oracle.dtw_features(X[:s], Y[:s], threads=threads)
        secs = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.dtw_features(X[:s], Y[:s])
        secs1 = time.perf_counter() - t0
        cpu = {"value": round(s * s / secs / 1e9, 5), "unit": "GCUPS", "cores": threads, "kind": "oracle",
               "sample": f"the leading {s}x{s} frames of the {n}x{m} pair (the whole pair would take "
                         f"{n * m / (s * s) * secs / 60:.0f} min on {threads} threads): FP64 cost rows + DP + "
                         f"int8 code matrix, the columns of each row split over {threads} threads, {secs:.2f} s",
               "single_thread": {"value": round(s * s / secs1 / 1e9, 5), "cores": 1, "seconds": round(secs1, 2)}}
        if not validate:
            return cpu, None
        # (1) The path is legal and its FP64 cost matches the FP32 total within
        # the FP32 rounding of the sweep: each step rounds a partial sum D_k
        # by at most 2^-24 D_k, and the partial sums along the path grow to
        # the total, so L steps stay within L 2^-25 of it on average (a
        # bound, loose; the measured gap is reported).
        # (2) Exactness at scale: a stretch of an optimal path is an optimal
        # path between its end cells (the cost of the rest of the path does
        # not depend on it), so the oracle is run on the sub-rectangles
        # between sampled pairs of path cells and must give the GPU's stretch,
        # up to declared ties. Ties are judged, as everywhere, on the full
        # problem's candidate totals: the sub-problem's plus D at the stretch's
        # first cell P less C(P), D(P) taken as the FP64 cost of the path's
        # prefix (the oracle's cost of the sub-pair from (0,0) to P).
        tol = parity.TOTAL_REL
        ok, msg, rescored, rel = True, "ok", None, None
        segments = []
        try:
            parity.check_legal(path, n, m)
            rescored = oracle.path_cost(X, Y, path)
            rel = abs(total - rescored) / abs(rescored)
            seg_len = 1500
            for q in np.linspace(0, len(path) - 1 - seg_len, 5).astype(np.int64):
                (pi, pj), (qi, qj) = path[q], path[q + seg_len]
                Xs, Ys = X[pi:qi + 1], Y[pj:qj + 1]
                _, BPs = oracle.dtw_features(Xs, Ys)
                sub = path[q:q + seg_len + 1] - np.array([pi, pj], dtype=path.dtype)
                parity.check_legal(sub, len(Xs), len(Ys))
                off = oracle.path_cost(X[:pi + 1], Y[:pj + 1], path[:q + 1]) - float(oracle.cost(Xs[:1], Ys[:1])[0, 0])
                ties = parity.audit_path(sub, BPs, lambda c, Xs=Xs, Ys=Ys, off=off:
                                         oracle.probe(c, X=Xs, Y=Ys)[0] + off)
                segments.append({"from": [int(pi), int(pj)], "to": [int(qi), int(qj)], "declared_ties": ties})
            msg = ("ok: path legal; 5 sampled stretches of 1500 steps equal the oracle's optimal paths between "
                   "their end cells; totals against the FP64 re-score of the path in total_within_1e-5 and "
                   "compensated_total_within_1e-5")
        except AssertionError as exc:
            ok, msg = False, str(exc)[:300]
        validation = {"path_legal_rescored_and_segments_exact": ok, "oracle_total": None,
                      "rescored_path_cost": rescored, "gpu_total": total, "rel_diff": rel, "rel_bound": tol,
                      "total_within_1e-5": bool(rel is not None and rel <= tol),
                      "compensated_total": comp,
                      "compensated_total_rel_err": (abs(comp - rescored) / rescored
                                                    if comp is not None and rescored else None),
                      "compensated_total_within_1e-5": (bool(abs(comp - rescored) <= tol * rescored)
                                                        if comp is not None and rescored else None),
                      "segments": segments, "path_len": int(len(path)), "detail": msg}
        return cpu, validation
    threads = host_threads()
    t0 = time.perf_counter()
    J, BP = oracle.dtw_features(X, Y, threads=threads)
    secs = time.perf_counter() - t0
    t0 = time.perf_counter()
    J1, BP1 = oracle.dtw_features(X, Y)
    secs1 = time.perf_counter() - t0
    same = (J1 == J) and np.array_equal(BP1, BP)
    del BP1
    cpu = {"value": round(n * m / secs / 1e9, 5), "unit": "GCUPS", "cores": threads, "kind": "oracle",
           "sample": f"the whole {n}x{m} pair: FP64 cost rows + DP + int8 code matrix, the columns of each row "
                     f"split over {threads} threads, {secs:.2f} s",
           "single_thread": {"value": round(n * m / secs1 / 1e9, 5), "cores": 1, "seconds": round(secs1, 2),
                             "bit_identical_to_threaded": bool(same)}}
    if not validate:
        return cpu, None
    ok, ties, msg = True, -1, "ok"
    try:
        parity.check_legal(path, n, m)
        parity.check_total(total, J)
        ties = parity.audit_path(path, BP, lambda c: oracle.probe(c, X=X, Y=Y)[0])
    except AssertionError as exc:  # report, do not hide
        ok, msg = False, str(exc)[:300]
    validation = {"path_match": ok, "declared_ties": ties, "oracle_total": J, "gpu_total": total,
                  "total_rel_err": abs(total - J) / J, "path_len": int(len(path)), "detail": msg}
    if comp is not None:
        # the compensated total (pardtw_path_total) against the oracle's optimum
        validation["compensated_total"] = comp
        validation["compensated_total_rel_err"] = abs(comp - J) / J
        validation["compensated_total_within_1e-5"] = bool(abs(comp - J) <= parity.TOTAL_REL * J)
    return cpu, validation


def cpu_baseline_batch(pairs, paths, totals, status, bf16=None, threads=8):
    """The oracle on every feasible pair of a batch (one thread per pair, a pool
    of `threads`), timed, then used to check the GPU paths (and, for the BF16
    form, to measure its cost error and re-score gap). The only use of the
    oracle in this script's batch mode."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    from tests import parity
    feas = [oracle.feasible(len(x), len(y)) for x, y in pairs]
    cells = sum(len(x) * len(y) for (x, y), f in zip(pairs, feas) if f)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        res = list(pool.map(lambda xy: oracle.dtw_features(*xy) if oracle.feasible(len(xy[0]), len(xy[1])) else None,
                            pairs))
    secs = time.perf_counter() - t0
    cpu = {"value": round(cells / secs / 1e9, 5), "unit": "GCUPS", "cores": threads, "kind": "oracle",
           "sample": f"all {len(pairs)} pairs ({cells:.3e} feasible cells), one pair per thread, {secs:.1f} s"}
    ok, ties, msg, devs = True, 0, "ok", []
    for b, (x, y) in enumerate(pairs):
        try:
            if not feas[b]:
                assert status[b] == 1 and len(paths[b]) == 0, "infeasible pair not reported"
                continue
            J, BP = res[b]
            parity.check_legal(paths[b], len(x), len(y))
            parity.check_total(float(totals[b]), J)
            ties += parity.audit_path(paths[b], BP, lambda c: oracle.probe(c, X=x, Y=y)[0])
            if bf16 is not None:
                p16, t16 = bf16[0][b], float(bf16[1][b])
                mdev, xdev = parity.path_deviation(p16, paths[b], len(x))
                devs.append((mdev, xdev, abs(t16 - J) / J, (oracle.path_cost(x, y, p16) - J) / J))
        except AssertionError as exc:
            ok, msg = False, f"pair {b}: {str(exc)[:200]}"
            break
    validation = {"path_match": ok, "declared_ties": ties, "detail": msg}
    if devs:
        a = np.array(devs)
        validation["bf16"] = {"mean_path_dev_frames": round(float(a[:, 0].mean()), 4),
                              "max_path_dev_frames": float(a[:, 1].max()),
                              "max_rel_cost_err": float(a[:, 2].max()),
                              "max_rescore_gap": float(a[:, 3].max())}
    return cpu, validation


# FP32 vector work per cell of the checkpointed sweep and of the backtrace's
# recomputed windows: three FMAs and two mins of the recurrence, and
# 1 - (acc * rx) * ry of the cost (whose dot product runs on MFMA)
CKPT_FLOPS_PER_CELL = 3 * 2 + 2 + 3
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak
# one compute unit's share of it: the one-workgroup backtrace
CU_FP32_PEAK_TFLOPS = FP32_PEAK_TFLOPS / 256


def ckpt_window_ranges(ie, je, r0):
    """The window the checkpointed backtrace recomputes for the block starting
    at row r0 entered at path cell (ie, je), with the kernel's own bounds: for
    each 64-column panel p, the 8-row chunks kbeg .. kend (rows r0 + 8k ..)
    where the cone je - 2(ie - r) <= c <= je - ceil((ie - r) / 2) meets it."""
    A = ie - r0
    cl = je - 2 * A - 2
    plo = cl // 64 if cl > 0 else 0
    out = []
    for p in range(plo, je // 64 + 1):
        over = je - (64 * p + 63)
        rmax = ie - (over + 1) // 2 if over > 0 else ie
        kend = (rmax - r0) // 8 if rmax >= r0 else -1
        rmin = ie - 2 * (je - 64 * p)
        kbeg = (rmin - r0) // 8 if rmin > r0 else 0
        out.append((p, kbeg, kend))
    return out


def ckpt_block_entries(path, n, K):
    """(r0, ie, je) for every block of K rows the path visits: the walk
    enters each block at its last path cell."""
    rows = path[:, 0].astype(np.int64)
    cols = path[:, 1].astype(np.int64)
    out = []
    for r0 in range(0, n, K):
        q = int(np.searchsorted(rows, r0 + K, side="left")) - 1  # rows ascend along the path
        if q >= 0 and rows[q] >= r0:
            out.append((r0, int(rows[q]), int(cols[q])))
    return out


def ckpt_window_cells(path, n, m, K):
    """Cells the checkpointed backtrace recomputes, from the path."""
    cells = 0
    for r0, ie, je in ckpt_block_entries(path, n, K):
        for p, kbeg, kend in ckpt_window_ranges(ie, je, r0):
            if kend >= kbeg:
                cells += (kend - kbeg + 1) * 8 * 64
    return cells


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU; runs on more than one GPU are not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_15478_amd import synth
    from paper_2607_15478_amd import pardtw as pd

    dev = torch.device("cuda:0")
    spec = synth.WORKLOADS[args.workload]
    assert spec["kind"] == "pair"
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    X, Y = synth.make_workload(args.workload)
    n, m, d = X.shape[0], Y.shape[0], X.shape[1]
    cells = n * m

    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    K = args.ckpt
    if K:
        w = pd.Workspace(n, m, dev, pd.LAYOUT_PANEL_BAND, cost=False, ckpt_rows=K)
    else:
        w = pd.Workspace(n, m, dev, pd.LAYOUT_PANEL_BAND, cost=not args.fused, packed=args.packed)
    stream = torch.cuda.current_stream()

    calib = None
    if args.calib_copy_gib > 0:
        nb = int(args.calib_copy_gib * (1 << 30))
        src = torch.empty(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"bytes_each_way": nb}
        del src, dst

    # Serial schedule (the default): cost, DP, split-walk backtrace and
    # compensated total of one pair, then the next. The split walk takes about
    # 0.1 ms at 50000 x 60000 (over checkpoints, a few ms at 600000 x 600000),
    # so hiding it buys less than the CUs it would take from the next pair's DP.
    # Pipelined schedule (--pipelined): the
    # cost and DP of each pair run on the launch stream, and the backtrace of
    # pair s (one workgroup) on a second stream beside the cost and DP of pair
    # s + 1. Pairs alternate between two workspaces; a workspace's codes are
    # written again only once the backtrace that reads them has finished.
    # (Running the cost GEMM of pair s + 1 beside the DP of pair s as well was
    # measured slower: the DP, a chain of waits across workgroups, lost more
    # than the GEMM saved.)
    # The checkpointed backtrace takes longer than its sweep, so there two
    # backtraces (of consecutive pairs, one workgroup each) run at once on
    # two streams, over three workspaces.
    # Extra workspaces are taken only as far as free device memory allows
    # (a 600000 x 600000 checkpointed pair needs 101 GB each); with none the
    # run is serial.
    pipelined = args.pipelined and not args.serial
    bufs = [w]
    if pipelined:
        per = sum(t.numel() * t.element_size() for t in (w.C, w.bp, w.ws, w.ckpt, w.path))
        free = torch.cuda.mem_get_info(dev)[0]
        extra = min(2 if K else 1, int(0.9 * free) // max(per, 1))
        for _ in range(extra):
            if K:
                bufs.append(pd.Workspace(n, m, dev, pd.LAYOUT_PANEL_BAND, cost=False, ckpt_rows=K))
            else:
                bufs.append(pd.Workspace(n, m, dev, pd.LAYOUT_PANEL_BAND, cost=not args.fused, packed=args.packed))
        pipelined = len(bufs) > 1
        bts = [torch.cuda.Stream(device=dev) for _ in range(len(bufs) - 1)]  # default priority
        side = (stream, bts)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        for b in bufs:
            pd.align_into(Xd, Yd, b, fused=args.fused or bool(K))
    torch.cuda.synchronize()

    if pipelined:
        return run_pair_pipelined(args, X, Y, Xd, Yd, bufs, stream, side, cells, calib)

    comp = not args.no_comp_total

    def one_step(e):
        """One pass of the hot path; e: four events around its stages, or None."""
        def rec(k):
            if e is not None:
                e[k].record(torch.cuda.current_stream())
        rec(0)
        if K:
            rec(1)
            pd.pardtw_dp_fused_ckpt(Xd, Yd, K, w.ckpt, w.total, w.status, w.ws)
            rec(2)
            if args.walk != "serial":
                pd.pardtw_ckpt_backtrace_parallel(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len, w.bt_ws)
            else:
                pd.pardtw_ckpt_backtrace(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len)
            if comp:
                pd.pardtw_path_total(Xd, Yd, w.path, w.path_len, w.total_comp, w.total_ws)
            rec(3)
            return
        if args.fused:
            rec(1)
            if args.packed:
                pd.pardtw_dp_fused_packed(Xd, Yd, w.bp, w.total, w.status, w.ws)
            else:
                pd.pardtw_dp_fused(Xd, Yd, w.bp, w.total, w.status, w.ws)
        else:
            pd.pardtw_cost(Xd, Yd, w.C, pd.PREC_F32, pd.LAYOUT_PANEL_BAND)
            rec(1)
            if args.packed:
                pd.pardtw_dp_packed(w.C, n, m, w.bp, w.total, w.status, w.ws, pd.LAYOUT_PANEL_BAND)
            else:
                pd.pardtw_dp(w.C, n, m, w.bp, w.total, w.status, w.ws, pd.LAYOUT_PANEL_BAND)
        rec(2)
        if args.walk != "serial":
            pd.pardtw_backtrace_parallel(w.bp, n, m, w.status, w.path, w.path_len, w.bt_ws, packed=args.packed)
        elif args.packed:
            pd.pardtw_backtrace_packed(w.bp, n, m, w.status, w.path, w.path_len)
        else:
            pd.pardtw_backtrace(w.bp, n, m, w.status, w.path, w.path_len)
        if comp:
            pd.pardtw_path_total(Xd, Yd, w.path, w.path_len, w.total_comp, w.total_ws)
        rec(3)

    graph = None
    if args.graph:
        # the whole step captured once as a hipGraph and replayed: one launch
        # per step instead of one host call per kernel (small pairs are
        # otherwise bound by the host issuing them); the stage times come from
        # eager steps before the timed region
        side = torch.cuda.Stream(device=dev)  # default priority
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            one_step(None)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            one_step(None)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(min(args.steps, 10))]
        for e in evs:
            one_step(e)
        torch.cuda.synchronize()
    else:
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    print(f"[bench] timing {args.steps} steps" + (" (graph replays)" if graph else ""), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if graph is not None:
        for _ in range(args.steps):
            graph.replay()
    else:
        for s in range(args.steps):
            one_step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(3)] for e in evs])
    cost_ms, dp_ms, bt_ms = stage_ms.mean(0)
    ms_per_step = wall * 1e3 / args.steps
    gcups = cells / (ms_per_step * 1e-3) / 1e9
    print(f"[bench] step {ms_per_step:.3f} ms (cost {cost_ms:.3f}, dp {dp_ms:.3f}, backtrace {bt_ms:.3f})",
          file=sys.stderr, flush=True)

    total = float(w.total.item())
    comp_total = None if args.no_comp_total else float(w.total_comp.item())
    L = int(w.path_len.item())
    path = w.path[:L].cpu().numpy()

    if K:
        out = ckpt_result(args, X, Y, path, total, cells, ms_per_step, cost_ms, dp_ms, bt_ms, w)
        print(json.dumps(out), flush=True)
        return

    roofline = pair_roofline(args, n, m, dp_ms)

    # ---- CPU baseline leg: the oracle on the whole pair, which also validates the GPU path ----
    cpu, validation = None, None
    if not args.no_cpu:
        cpu, validation = cpu_baseline_pair(X, Y, path, total, validate=not args.no_validate,
                                            comp=comp_total)

    out = {
        "metric": "DP cells/sec (GCUPS) + aligned pairs/sec at oracle path match, 1 MI355X",
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "d": d, "cells": cells,
                   "layout": ("fused_cost" if args.fused else "panel64_band") + ("+packed_codes" if args.packed else ""),
                   "device_bytes_per_pair": workspace_device_bytes(w),
                   "device_bytes_per_cell": round(workspace_device_bytes(w) / cells, 4),
                   "schedule": "serial: cost, DP and backtrace of one pair, then the next"
                               + (", each step one hipGraph replay" if args.graph else ""),
                   "walk": "one workgroup" if args.walk == "serial" else "split",
                   "pairs_per_s": round(1e3 / ms_per_step, 3),
                   "stage_ms": {"cost": round(float(cost_ms), 4), "dp": round(float(dp_ms), 4),
                                "backtrace": round(float(bt_ms), 4)}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "validation": validation,
    }
    if calib:
        out["calibration_copy"] = calib
    print(json.dumps(out), flush=True)


def launch_pipelined(pd, Xd, Yd, bufs, stream, side, steps, fused, K, evs, after_bt=None, serial_walk=False):
    """Enqueue `steps` pairs in the pipelined schedule: cost (materialised
    form) and DP on `stream`, each backtrace on one of the backtrace streams
    side[1] (in turn) once its DP is done. Pair s uses workspace
    bufs[s % len(bufs)]; its cost matrix and codes (or checkpoints) are
    rewritten only after the DP and the backtrace of the pair before that
    read them. evs[s] holds six events: cost start/end, DP start/end,
    backtrace start/end. after_bt(s, w, s_bt) may enqueue work on the
    backtrace stream after pair s's backtrace, before its end event."""
    n, m = Xd.shape[0], Yd.shape[0]
    s_cost, bts = side
    nb = len(bufs)
    for s in range(steps):
        e = evs[s]
        w = bufs[s % nb]
        s_bt = bts[s % len(bts)]
        if not fused and not K:
            if s >= nb:
                s_cost.wait_event(evs[s - nb][3])  # the DP that read this cost matrix
            e[0].record(s_cost)
            pd.pardtw_cost(Xd, Yd, w.C, pd.PREC_F32, pd.LAYOUT_PANEL_BAND, stream=s_cost)
            e[1].record(s_cost)
            stream.wait_event(e[1])
        if s >= nb:
            stream.wait_event(evs[s - nb][5])  # the backtrace that read these codes
        e[2].record(stream)
        if K:
            pd.pardtw_dp_fused_ckpt(Xd, Yd, K, w.ckpt, w.total, w.status, w.ws, stream=stream)
        elif fused and w.packed:
            pd.pardtw_dp_fused_packed(Xd, Yd, w.bp, w.total, w.status, w.ws, stream=stream)
        elif fused:
            pd.pardtw_dp_fused(Xd, Yd, w.bp, w.total, w.status, w.ws, stream=stream)
        elif w.packed:
            pd.pardtw_dp_packed(w.C, n, m, w.bp, w.total, w.status, w.ws, pd.LAYOUT_PANEL_BAND, stream=stream)
        else:
            pd.pardtw_dp(w.C, n, m, w.bp, w.total, w.status, w.ws, pd.LAYOUT_PANEL_BAND, stream=stream)
        e[3].record(stream)
        s_bt.wait_event(e[3])
        e[4].record(s_bt)
        if K and not serial_walk:
            pd.pardtw_ckpt_backtrace_parallel(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len, w.bt_ws, stream=s_bt)
        elif K:
            pd.pardtw_ckpt_backtrace(Xd, Yd, K, w.ckpt, w.status, w.path, w.path_len, stream=s_bt)
        elif not serial_walk:
            pd.pardtw_backtrace_parallel(w.bp, n, m, w.status, w.path, w.path_len, w.bt_ws, stream=s_bt,
                                         packed=w.packed)
        elif w.packed:
            pd.pardtw_backtrace_packed(w.bp, n, m, w.status, w.path, w.path_len, stream=s_bt)
        else:
            pd.pardtw_backtrace(w.bp, n, m, w.status, w.path, w.path_len, stream=s_bt)
        if after_bt is not None:
            after_bt(s, w, s_bt)
        e[5].record(s_bt)


def run_pair_pipelined(args, X, Y, Xd, Yd, bufs, stream, side, cells, calib):
    """K pairs back to back: cost and DP on the launch stream, each pair's
    backtrace on a second stream beside the next pair's cost and DP (see
    main; `side` is the cost stream, here the launch stream, and the
    backtrace stream). Every step's cost, DP and backtrace run inside the
    timed region."""
    import torch
    from paper_2607_15478_amd import pardtw as pd
    n, m, d = X.shape[0], Y.shape[0], X.shape[1]
    K = args.ckpt
    # per step: cost start/end, DP start/end, backtrace start/end
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    print(f"[bench] timing {args.steps} pipelined steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    after = None
    if not args.no_comp_total:
        def after(s, w, s_bt):
            pd.pardtw_path_total(Xd, Yd, w.path, w.path_len, w.total_comp, w.total_ws, stream=s_bt)
    launch_pipelined(pd, Xd, Yd, bufs, stream, side, args.steps, args.fused, K, evs, after_bt=after,
                     serial_walk=args.walk != "split")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = np.array([[0.0 if (args.fused or K) else e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3]),
                          e[4].elapsed_time(e[5])] for e in evs])
    cost_ms, dp_ms, bt_ms = stage_ms.mean(0)
    ms_per_step = wall * 1e3 / args.steps
    gcups = cells / (ms_per_step * 1e-3) / 1e9
    print(f"[bench] step {ms_per_step:.3f} ms pipelined (cost {cost_ms:.3f}, dp {dp_ms:.3f}, backtrace {bt_ms:.3f} "
          f"on its own stream)", file=sys.stderr, flush=True)
    layout = (f"pipelined: each pair's backtrace on one of {len(side[1])} backtrace stream(s) beside the next "
              f"pairs' {'sweeps' if K else 'cost and DP'}, {len(bufs)} workspaces in turn (--serial: one after another)")
    w = bufs[(args.steps - 1) % len(bufs)]
    total = float(w.total.item())
    comp_total = None if args.no_comp_total else float(w.total_comp.item())
    L = int(w.path_len.item())
    path = w.path[:L].cpu().numpy()
    if K:
        out = ckpt_result(args, X, Y, path, total, cells, ms_per_step, cost_ms, dp_ms, bt_ms, w)
        out["config"]["schedule"] = layout
        out["config"]["latency_ms"] = round(float(dp_ms + bt_ms), 4)
        print(json.dumps(out), flush=True)
        return
    roofline = pair_roofline(args, n, m, dp_ms)
    cpu, validation = None, None
    if not args.no_cpu:
        cpu, validation = cpu_baseline_pair(X, Y, path, total, validate=not args.no_validate,
                                            comp=comp_total)
    out = {
        "metric": "DP cells/sec (GCUPS) + aligned pairs/sec at oracle path match, 1 MI355X",
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "d": d, "cells": cells,
                   "layout": ("fused_cost" if args.fused else "panel64_band") + ("+packed_codes" if args.packed else ""),
                   "device_bytes_per_pair": workspace_device_bytes(bufs[0]),
                   "device_bytes_per_cell": round(workspace_device_bytes(bufs[0]) / cells, 4),
                   "schedule": layout,
                   "walk": "split" if args.walk == "split" else "one workgroup",
                   "pairs_per_s": round(1e3 / ms_per_step, 3),
                   "latency_ms": round(float(cost_ms + dp_ms + bt_ms), 4),
                   "stage_ms": {"cost": round(float(cost_ms), 4), "dp": round(float(dp_ms), 4),
                                "backtrace": round(float(bt_ms), 4)}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "validation": validation,
    }
    if calib:
        out["calibration_copy"] = calib
    print(json.dumps(out), flush=True)


_COPY = {}


def copy_bandwidth():
    """Bandwidth of a plain device-to-device copy (torch copy_, 1 GiB each
    way, larger than the 256 MB Infinity Cache), bytes read + written per
    second, measured once per process beside the datasheet peak; None when
    less than 3 GiB of device memory is free."""
    import torch
    if "v" not in _COPY:
        free, _ = torch.cuda.mem_get_info()
        nb = 1 << 30
        if free < 3 * nb:
            _COPY["v"] = None
        else:
            src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                dst.copy_(src)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            _COPY["v"] = {"GBps": round(2 * nb / (ms * 1e-3) / 1e9, 1), "bytes_each_way": nb, "ms": round(ms, 4)}
            del src, dst
            torch.cuda.empty_cache()
    return _COPY["v"]


def pair_roofline(args, n, m, dp_ms):
    """The DP kernel against the HBM peak. Algorithmic bytes are those of the
    method's own work, the path band (cells on some path from (0,0) to
    (n-1,m-1)): 4 B of cost read and 1 B of code written per band cell (1 B
    with the fused cost). The dense all-cells figure is reported only under
    its own label. `traffic` is the counter-measured bytes of one launch when
    the counters were taken on this DP source."""
    # 4 B of cost read (none when fused), 1 B of code written (2 bits packed)
    bpc = (0 if args.fused else DP_BYTES_PER_CELL - 1) + (0.25 if args.packed else 1)
    bcells = band_cells(n, m)
    alg = bpc * bcells
    dp_achieved = alg / (dp_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            src = open(os.path.join(ROOT, "paper_2607_15478_amd", "csrc", "dp.hip"), "rb").read()
            if (not args.fused and not args.packed and tj.get("workload") == args.workload
                    and tj.get("dp_source_sha256") == hashlib.sha256(src).hexdigest()):
                traffic = tj.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    dense = bpc * n * m / (dp_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(dp_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dp_achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "dp_kernel" + (" (fused cost)" if args.fused else "") + (" (packed codes)" if args.packed else ""),
                "algorithmic_bytes_per_launch": int(alg), "bytes_per_band_cell": bpc, "band_cells": bcells,
                "band_fraction": round(bcells / (n * m), 4), "kernel_ms": round(float(dp_ms), 4),
                "dense_equivalent": {"note": "all n*m cells at the same bytes per cell; not the method's work",
                                     "GBps": round(dense, 1), "frac": round(dense / HBM_PEAK_GBS, 4)}}
    if traffic:
        roofline["traffic_over_algorithmic"] = round(traffic / alg, 3)
        roofline["moved_GBps"] = round(traffic / (dp_ms * 1e-3) / 1e9, 1)
    roofline["measured_copy"] = copy_bandwidth()
    return roofline


def ckpt_result(args, X, Y, path, total, cells, ms_per_step, cost_ms, dp_ms, bt_ms, w):
    """The bench line of the checkpointed path. Both its kernels do FP32
    vector work on cells (the sweep on the path band, the backtrace on its
    recomputed windows), with no HBM traffic to speak of (no cost matrix, no
    codes), so each is set against the FP32 vector peak: the whole chip's, or
    one compute unit's share for the one-workgroup walk. `roofline` names the
    longer of the two and carries the other."""
    from paper_2607_15478_amd import pardtw as pd
    n, m, d = X.shape[0], Y.shape[0], X.shape[1]
    K = args.ckpt
    bcells = band_cells(n, m)
    sweep_ach = bcells * CKPT_FLOPS_PER_CELL / (dp_ms * 1e-3) / 1e12
    sweep = {"bound": "alu", "achieved": round(sweep_ach, 4), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": round(sweep_ach / FP32_PEAK_TFLOPS, 4), "traffic": None,
             "kernel": "dp_kernel (fused cost, checkpoints)", "band_cells": bcells,
             "flops_per_cell": CKPT_FLOPS_PER_CELL, "kernel_ms": round(float(dp_ms), 4),
             "note": "chain-bound: rows of a panel in sequence, panels in a staircase"}
    wcells = ckpt_window_cells(path, n, m, K)
    one_wg = args.walk == "serial"
    bt_peak = CU_FP32_PEAK_TFLOPS if one_wg else FP32_PEAK_TFLOPS
    bt_ach = wcells * CKPT_FLOPS_PER_CELL / (bt_ms * 1e-3) / 1e12
    bt = {"bound": "alu", "achieved": round(bt_ach, 5), "peak": round(bt_peak, 4),
          "unit": "TFLOP/s", "frac": round(bt_ach / bt_peak, 4), "traffic": None,
          "kernel": "ckpt_backtrace_kernel" if one_wg else "ck_seg_round_kernel (split walk)",
          "peak_scope": "one CU (the kernel is one workgroup)" if one_wg else "the chip",
          "window_cells_per_launch": wcells, "flops_per_cell": CKPT_FLOPS_PER_CELL,
          "kernel_ms": round(float(bt_ms), 4)}
    if dp_ms >= bt_ms:
        roofline = dict(sweep, backtrace=bt)
    else:
        roofline = dict(bt, sweep=sweep)
    comp_total = None if args.no_comp_total else float(w.total_comp.item())
    cpu, validation = None, None
    if not args.no_cpu:
        cpu, validation = cpu_baseline_pair(X, Y, path, total, validate=not args.no_validate,
                                            comp=comp_total)
    gcups = cells / (ms_per_step * 1e-3) / 1e9
    return {
        "metric": "DP cells/sec (GCUPS) + aligned pairs/sec at oracle path match, 1 MI355X",
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "d": d, "cells": cells,
                   "layout": "checkpointed", "rows_per_block": K,
                   "schedule": "serial: sweep and backtrace of one pair, then the next",
                   "walk": "one workgroup" if args.walk == "serial" else "split",
                   "checkpoint_bytes": pd.pardtw_ckpt_bytes(n, m, K),
                   "device_bytes_per_pair": workspace_device_bytes(w),
                   "device_bytes_per_cell": round(workspace_device_bytes(w) / cells, 4),
                   "code_matrix_bytes_avoided": pd.pardtw_bp_bytes(n, m),
                   "pairs_per_s": round(1e3 / ms_per_step, 3),
                   "stage_ms": {"dp_ckpt": round(float(dp_ms), 4), "backtrace_ckpt": round(float(bt_ms), 4)}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "validation": validation,
    }


def run_batch(args):
    """Batched form: every pair of a batch workload in one hipGraph replay of
    pardtw_align_batch (autotuned schedule), against the same pairs aligned by
    sequential single-pair calls. For the D = 128 workload the BF16-cost form is
    run too and its paths compared with the FP32 ones."""
    import torch
    from paper_2607_15478_amd import synth
    from paper_2607_15478_amd import pardtw as pd

    dev = torch.device("cuda:0")
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    pairs = synth.make_workload(args.workload)
    ns, ms = [len(p[0]) for p in pairs], [len(p[1]) for p in pairs]
    d = pairs[0][0].shape[1]
    feas = [(n - 1) <= 2 * (m - 1) and (m - 1) <= 2 * (n - 1) for n, m in zip(ns, ms)]
    cells = sum(n * m for n, m, f in zip(ns, ms, feas) if f)

    Xp, Yp = pd.pack(pairs, dev)
    res = {}
    for prec in ([pd.PREC_F32, pd.PREC_BF16] if d >= 64 else [pd.PREC_F32]):
        # fused: FP32 costs for d <= 16, BF16-operand costs for d <= 128 (d % 8 == 0)
        fusable = (d <= 16) if prec == pd.PREC_F32 else (d <= 128 and d % 8 == 0)
        # FP32 d <= 16 fuses by default (faster on the batches); BF16 on request
        want = args.fused or (prec == pd.PREC_F32 and not args.materialised)
        plan = pd.Plan(ns, ms, d, prec, fused=want and fusable)
        buf = plan.buffers(dev)
        best = plan.autotune(Xp, Yp, buf, reps=2)
        for _ in range(args.warmup):
            plan.align(Xp, Yp, buf)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.align(Xp, Yp, buf)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            plan.align(Xp, Yp, buf)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / args.steps
        res[prec] = dict(plan=plan, buf=buf, ms=ms_graph, tuned_dp_ms=best, sched=plan.schedule(),
                         fused=bool(want and fusable),
                         totals=buf["totals"].cpu().numpy(), status=buf["status"].cpu().numpy(),
                         paths=[plan.path(buf, b).cpu().numpy() for b in range(len(pairs))])
        print(f"[bench] batch prec={prec} graph {ms_graph:.3f} ms, schedule {plan.schedule()}", file=sys.stderr,
              flush=True)

    # forward + backward of the differentiable form (the D = 128 workload):
    # one graph replay of pardtw_align_batch + pardtw_path_grad_batch, and
    # the backward alone with HIP events
    fwd_bwd = None
    if d >= 64:
        fwd_bwd = time_forward_backward(torch, res[pd.PREC_F32]["plan"], res[pd.PREC_F32]["buf"], Xp, Yp,
                                        args.steps)
        print(f"[bench] forward+backward graph {fwd_bwd['graph_ms']:.3f} ms, backward {fwd_bwd['grad_ms']:.4f} ms",
              file=sys.stderr, flush=True)

    # sequential single-pair calls on preallocated workspaces
    ws = [pd.Workspace(n, m, dev) for n, m in zip(ns, ms)]
    Xs = [torch.from_numpy(x).to(dev) for x, _ in pairs]
    Ys = [torch.from_numpy(y).to(dev) for _, y in pairs]
    for b in range(len(pairs)):
        pd.align_into(Xs[b], Ys[b], ws[b])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for b in range(len(pairs)):
        pd.align_into(Xs[b], Ys[b], ws[b])
    e1.record()
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1)
    r32 = res[pd.PREC_F32]
    same_as_single = all(
        (not feas[b]) or (np.array_equal(r32["paths"][b], ws[b].path[: int(ws[b].path_len.item())].cpu().numpy())
                          and float(r32["totals"][b]) == float(ws[b].total.item()))
        for b in range(len(pairs)))
    del ws

    # ---- CPU baseline leg: the oracle on every pair, which also validates the GPU paths ----
    cpu, validation = None, None
    if not args.no_cpu:
        bf16 = None
        if pd.PREC_BF16 in res:
            bf16 = (res[pd.PREC_BF16]["paths"], res[pd.PREC_BF16]["totals"])
        cpu, validation = cpu_baseline_batch(pairs, r32["paths"], r32["totals"], r32["status"], bf16,
                                             threads=min(8, host_threads()))
        validation["batch_equals_single_pair_calls"] = same_as_single
        if fwd_bwd is not None:
            gcpu, gval = cpu_baseline_grad(pairs, r32["paths"], fwd_bwd)
            cpu["backward"] = gcpu
            validation["gradient"] = gval

    out = {
        "metric": "DP cells/sec (GCUPS) + aligned pairs/sec at oracle path match, 1 MI355X",
        "value": round(cells / (r32["ms"] * 1e-3) / 1e9, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "pairs": len(pairs), "feasible_pairs": int(sum(feas)), "d": d,
                   "feasible_cells": cells, "pairs_per_s": round(len(pairs) / (r32["ms"] * 1e-3), 1),
                   "schedule": r32["sched"], "tuned_dp_ms": round(r32["tuned_dp_ms"], 4),
                   "sequential_single_pair_ms": round(ms_seq, 3),
                   "speedup_vs_sequential": round(ms_seq / r32["ms"], 2)},
        "cpu_baseline": cpu,
        "validation": validation,
    }
    if pd.PREC_BF16 in res:
        out["config"]["bf16_graph_ms"] = round(res[pd.PREC_BF16]["ms"], 4)
    if fwd_bwd is not None:
        out["config"]["forward_backward_graph_ms"] = round(fwd_bwd["graph_ms"], 4)
        out["config"]["backward_ms"] = round(fwd_bwd["grad_ms"], 4)
    # the dominant kernel, the batched DP, on the pairs' path bands (tuned
    # time); with the fused cost it reads no costs, only writes its codes
    bcells = sum(band_cells(n, m) for n, m, f in zip(ns, ms, feas) if f)
    dp_ms = r32["tuned_dp_ms"]
    bpc = 1 if r32["fused"] else DP_BYTES_PER_CELL
    ach = bpc * bcells / (dp_ms * 1e-3) / 1e9
    out["config"]["fused_cost"] = r32["fused"]
    out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                       "kernel": "dp_batch_kernel (fused cost)" if r32["fused"] else "dp_batch_kernel",
                       "algorithmic_bytes_per_launch": bpc * bcells, "bytes_per_band_cell": bpc,
                       "band_cells": bcells, "kernel_ms": round(dp_ms, 4), "measured_copy": copy_bandwidth()}
    print(json.dumps(out), flush=True)


def time_forward_backward(torch, plan, buf, Xp, Yp, steps):
    """Forward (pardtw_align_batch) + backward (pardtw_path_grad_batch, dL/dJ
    = 1 per pair) of the batch: one graph replay per step, and the backward
    kernel alone timed with HIP events on the launch stream. Returns the
    timings and the gradients of the last replay."""
    g = torch.ones(plan.batch, dtype=torch.float32, device=Xp.device)
    dX, dY = torch.empty_like(Xp), torch.empty_like(Yp)
    plan.align(Xp, Yp, buf)
    plan.path_grad(Xp, Yp, buf, g, dX, dY)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.align(Xp, Yp, buf)
        plan.path_grad(Xp, Yp, buf, g, dX, dY)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        plan.align(Xp, Yp, buf)
        plan.path_grad(Xp, Yp, buf, g, dX, dY)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(steps):
        plan.path_grad(Xp, Yp, buf, g, dX, dY)
    e1.record(stream)
    torch.cuda.synchronize()
    grad_ms = e0.elapsed_time(e1) / steps
    return {"graph_ms": graph_ms, "grad_ms": grad_ms, "dX": dX.cpu().numpy(), "dY": dY.cpu().numpy(),
            "x_off": list(plan.x_off), "y_off": list(plan.y_off)}


def cpu_baseline_grad(pairs, paths, fb):
    """The oracle's FP64 fixed-path gradient of every pair, timed on one host
    thread, against the GPU's backward (dL/dJ = 1). The only use of the
    oracle for the backward."""
    import oracle
    t0 = time.perf_counter()
    ref = [oracle.path_grad(x, y, p, 1.0) if len(p) else None for (x, y), p in zip(pairs, paths)]
    secs = time.perf_counter() - t0
    worst = 0.0
    for b, ((x, y), r) in enumerate(zip(pairs, ref)):
        if r is None:
            continue
        gx = fb["dX"][fb["x_off"][b]: fb["x_off"][b] + len(x)]
        gy = fb["dY"][fb["y_off"][b]: fb["y_off"][b] + len(y)]
        scale = max(np.abs(r[0]).max(), np.abs(r[1]).max())
        worst = max(worst, float(np.abs(gx - r[0]).max()) / scale, float(np.abs(gy - r[1]).max()) / scale)
    rows = sum(len(p) for p in paths)
    cpu = {"value": round(rows / secs, 1), "unit": "path cells/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 fixed-path gradient of all {len(pairs)} pairs ({rows} path cells), one thread, "
                     f"{secs:.2f} s"}
    return cpu, {"max_abs_err_over_max_grad": float(worst), "within_1e-4": bool(worst <= 1e-4)}


def path_rows_position(path, n: int) -> np.ndarray:
    """For each row i < n of A, the mean column of B the path visits in that
    row, linearly interpolated over rows it skips (a (2,1) step skips one) and
    held constant before its first and after its last row."""
    path = np.asarray(path, np.int64).reshape(-1, 2)
    s, c = np.zeros(n), np.zeros(n)
    np.add.at(s, path[:, 0], path[:, 1])
    np.add.at(c, path[:, 0], 1)
    have = c > 0
    rows = np.arange(n)
    return np.interp(rows, rows[have], s[have] / c[have])


def path_deviation(path, ref_path, n: int) -> dict:
    """Deviation in frames of `path` from `ref_path`, both over the n rows of
    A: mean and max over rows i of |j(i) - j_ref(i)| (path_rows_position), and
    the share of rows within 1 and 10 frames."""
    dev = np.abs(path_rows_position(path, n) - path_rows_position(ref_path, n))
    return {"mean_dev_frames": round(float(dev.mean()), 4), "max_dev_frames": round(float(dev.max()), 2),
            "rows_within_1_frame": round(float((dev <= 1.0).mean()), 5),
            "rows_within_10_frames": round(float((dev <= 10.0).mean()), 5)}


def cpu_baseline_segmental(A, B, starts, hop, variant, g_S, g_ends, g_total, sample_frags):
    """The oracle's subsequence DP timed on a bounded sample of fragments (their
    scores then checked against the GPU's), and the oracle's segment level run
    on the GPU's own scores (ends and total checked). The only use of the
    oracle in this script's segmental mode."""
    import oracle
    from tests import parity
    cells, t_dp = 0, 0.0
    worst = 0.0
    for f in sample_frags:
        x = A[starts[f]:starts[f + 1]]
        t0 = time.perf_counter()
        S, _ = oracle.subseq_features(x, B)
        t_dp += time.perf_counter() - t0
        cells += len(x) * len(B)
        fin = np.isfinite(S)
        ok_inf = np.array_equal(np.isfinite(g_S[f]), fin)
        rel = np.abs(g_S[f][fin].astype(np.float64) - S[fin]) / np.maximum(np.abs(S[fin]), 1e-30)
        worst = max(worst, float(rel.max()) if rel.size else 0.0, 0.0 if ok_inf else np.inf)
    cpu = {"value": round(cells / t_dp / 1e9, 5), "unit": "GCUPS", "cores": 1, "kind": "oracle",
           "sample": f"fragments {list(sample_frags)}: FP64 cost rows + subsequence DP + int8 codes over the whole "
                     f"reference, one thread, {cells:.3e} cells in {t_dp:.1f} s"}
    total, ends = oracle.segment_ends(g_S.astype(np.float64), hop, variant)
    got = float(np.sum(g_S.astype(np.float64)[np.arange(len(g_ends)), g_ends])) if np.all(g_ends >= 0) else np.inf
    validation = {"sampled_scores_max_rel_err": worst, "scores_within_1e-5": worst <= parity.TOTAL_REL,
                  "ends_equal_oracle_on_gpu_scores": bool(np.array_equal(ends, g_ends)),
                  "placement_within_tie_tolerance": bool(got <= total * (1 + parity.TIE_REL) + 1e-9),
                  "oracle_total": total, "gpu_total": g_total}
    return cpu, validation


def run_segmental(args):
    """Segmental DTW (NSDTW or WSDTW) of one long pair: one hipGraph replay of
    pardtw_segmental_align = fragment cost GEMMs -> one persistent subsequence
    DP over every fragment -> segment level -> fragment backtraces ->
    concatenation. GCUPS counts the whole la x lb matrix, which the fragments
    tile exactly."""
    import torch
    from paper_2607_15478_amd import synth
    from paper_2607_15478_amd import pardtw as pd

    dev = torch.device("cuda:0")
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    A, B = synth.make_workload(args.workload)
    la, lb, d = A.shape[0], B.shape[0], A.shape[1]
    nf, variant = args.nfrag, (pd.WSDTW if args.variant == "wsdtw" else pd.NSDTW)
    cells = la * lb
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    fused = (args.fused or not args.materialised) and d <= 16
    plan = pd.SegPlan(la, lb, nf, d, pd.PREC_F32, variant, fused=fused)
    buf = plan.buffers(dev)
    print(f"[bench] plan {nf} fragments, workspace {plan.workspace_bytes / 2**30:.1f} GiB; autotune",
          file=sys.stderr, flush=True)
    dp_ms = plan.autotune(Ad, Bd, buf, reps=2)
    for _ in range(args.warmup):
        plan.align(Ad, Bd, buf)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.align(Ad, Bd, buf)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.align(Ad, Bd, buf)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} graph replays", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = e0.elapsed_time(e1) / args.steps
    print(f"[bench] segmental {ms:.3f} ms per alignment (DP {dp_ms:.3f} ms)", file=sys.stderr, flush=True)

    g_S = plan.scores(buf).cpu().numpy()
    g_ends = buf["ends"].cpu().numpy().astype(np.int64)
    g_total = float(buf["total"].item())
    L = int(buf["path_len"].item())
    seg_path = buf["path"][:L].cpu().numpy()
    seg_status = int(buf["status"].item())
    # Accuracy against exact DTW of the same pair (outside the timed region):
    # the segmental path's deviation from the exact path, row by row of A.
    accuracy = None
    if not args.no_accuracy:
        w = pd.Workspace(la, lb, "cuda", pd.LAYOUT_PANEL_BAND, cost=False, packed=True)
        pd.align_into(Ad, Bd, w, fused=True)
        torch.cuda.synchronize()
        if int(w.status.item()) == pd.PAIR_OK:
            exact = w.path[: int(w.path_len.item())].cpu().numpy()
            accuracy = {"reference": "exact DTW path of the same pair (weights 2,3,3)",
                        **path_deviation(seg_path, exact, la)}
        del w
    bpc = 1 if fused else DP_BYTES_PER_CELL
    # the method's work: each fragment's subsequence band (cells on some path
    # from its first row to its last)
    bcells = sum(subseq_band_cells(plan.starts[f + 1] - plan.starts[f], lb) for f in range(nf))
    dp_achieved = bpc * bcells / (dp_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(dp_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dp_achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": ("frag_sweep_kernel (%d waves per fragment)" % plan.schedule()["waves"]
                           if plan.schedule()["panels_per_workgroup"] == 0 else
                           "dp_batch_kernel (subsequence%s)" % (", fused cost" if fused else "")),
                "algorithmic_bytes_per_launch": bpc * bcells, "bytes_per_band_cell": bpc, "band_cells": bcells,
                "band_fraction": round(bcells / cells, 4), "kernel_ms": round(float(dp_ms), 4),
                "measured_copy": copy_bandwidth()}
    cpu, validation = None, None
    if not args.no_cpu:
        # a bounded sample: up to three fragments, at most 3e9 cells (about 15 s on one core)
        sample, used = [], 0
        for f in sorted({0, nf // 2, nf - 1}):
            c = (plan.starts[f + 1] - plan.starts[f]) * lb
            if used + c <= 3e9:
                sample.append(f)
                used += c
        if sample:
            cpu, validation = cpu_baseline_segmental(A, B, plan.starts, plan.hop, variant, g_S, g_ends, g_total,
                                                     sample)
    out = {
        "metric": "DP cells/sec (GCUPS) + aligned pairs/sec at oracle path match, 1 MI355X",
        "value": round(cells / (ms * 1e-3) / 1e9, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "algorithm": args.variant, "fragments": nf, "hop": plan.hop,
                   "fused_cost": fused, "workspace_gib": round(plan.workspace_bytes / 2**30, 2),
                   "la": la, "lb": lb, "d": d, "cells": cells, "pairs_per_s": round(1e3 / ms, 3),
                   "wall_ms_per_step": round(wall, 4), "schedule": plan.schedule(), "tuned_dp_ms": round(dp_ms, 4),
                   "status": seg_status, "path_len": L},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "validation": validation,
        "accuracy": accuracy,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    _wl = sys.argv[sys.argv.index("--workload") + 1] if "--workload" in sys.argv[:-1] else ""
    if _wl.startswith("batch") or _wl.startswith("segmental"):
        _a = parse()
        if _a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
            print("bench.py: measures one GPU; runs on more than one GPU are not supported", file=sys.stderr)
            sys.exit(2)
        run_batch(_a) if _wl.startswith("batch") else run_segmental(_a)
    else:
        main()
