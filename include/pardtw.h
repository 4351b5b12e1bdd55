/*
 * pardtw.h -- C ABI of libpardtw.so: exact Parallelized Diagonal DTW (ParDTW)
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Yang, Shaw & Tsai, "A Study of Parallelizable Alternatives to Dynamic
 * Time Warping for Aligning Long Sequences". Given two feature sequences the
 * library returns the optimal DTW alignment path (a sequence of coordinate
 * pairs) and its cost (problem statement: Sec. I; outputs: Sec. VI-D).
 *
 *   cost     C[i,j] = 1 - <x_i, y_j> / (|x_i| |y_j|)   (cosine distance, Sec. IV)
 *   DP       steps (1,1), (1,2), (2,1) with weights 2, 3, 3 (Sec. V); the weight
 *            multiplies the cost of the cell a step lands on; D[0,0] = C[0,0];
 *            D[i,j] = min(D[i-1,j-1] + 2C, D[i-1,j-2] + 3C, D[i-2,j-1] + 3C)
 *   codes    0 = (1,1), 1 = (1,2), 2 = (2,1), 3 = origin; an exact tie goes to
 *            the lowest code. Four codes = the paper's 2-bit transition types
 *            (Sec. VI-D). pardtw_dp defines them on the band of cells that can
 *            lie on a path from (0,0) to (N-1,M-1); the optimal path and every
 *            cell the backtrace reads lie in it.
 *   result   D[N-1, M-1] and the path from (0,0) to (N-1,M-1), exactly DTW's
 *            (Sec. II-D: ParDTW changes the order of work, not the result).
 *
 * Conventions. X is N x d (rows i, the query), Y is M x d (columns j, the
 * reference); both row-major FP32. Sizes are int64, coordinates int32. Every
 * pointer argument named "device" must point to GPU memory owned by the caller;
 * the library allocates no memory in these calls (plans are the only
 * library-owned objects and are created ahead of time). All calls are
 * asynchronous on the given stream and never synchronise it.
 *
 * Errors. The return value reports host-side argument validation and launch
 * errors only. Per-pair outcomes are written to a device int32 status:
 * PARDTW_PAIR_OK, or PARDTW_PAIR_INFEASIBLE when no legal path exists
 * (M-1 > 2(N-1) or N-1 > 2(M-1)); an infeasible pair gets total = +inf and
 * path_len = 0.
 */
#ifndef PARDTW_H
#define PARDTW_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PARDTW_OK = 0,
    PARDTW_ERR_INVALID_ARG = 1, /* null pointer, non-positive or overflowing size */
    PARDTW_ERR_WORKSPACE = 2,   /* workspace missing or smaller than required */
    PARDTW_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed */
    PARDTW_ERR_UNSUPPORTED = 4  /* combination not implemented (e.g. bad layout) */
} pardtw_status;

typedef enum {
    PARDTW_PREC_F32 = 0,  /* FP32 features, FP32 MFMA products, FP32 accumulation */
    PARDTW_PREC_BF16 = 1  /* features rounded to BF16 for the MFMA GEMM, FP32 accumulation */
} pardtw_prec;

typedef enum {
    /* Row-major N x M: C[i*M + j]. */
    PARDTW_LAYOUT_ROW = 0,
    /* Column panels of 64 columns, each cut into groups of 8 rows; a group
     * stores rows 0-3 of its 64 columns, then rows 4-7, each column's 4 rows
     * contiguous:
     *   C[((p*G + i/8)*2 + (i%8)/4)*256 + (j - 64p)*4 + i%4],
     *   p = j/64, G = ceil(N/8), P = ceil(M/64) panels, P*G*512 floats.
     * Columns past M and rows past N are padding. A wavefront of the DP reads
     * one 8-row chunk of its panel with two 1 KB contiguous loads. */
    PARDTW_LAYOUT_PANEL = 1,
    /* The panel layout with only the 8-row groups that pardtw_dp reads: the
     * band of cells that can lie on a path from (0,0) to (N-1,M-1) with the
     * step set of Sec. V. A group of panel p is written when it holds a real
     * cell reachable from the origin (j <= 2i and i <= 2j) and a real cell
     * from which (N-1,M-1) is reachable ((M-1-j) <= 2(N-1-i) and
     * (N-1-i) <= 2(M-1-j)); for 64p <= 2(N-1), j1 = min(64p+63, M-1):
     *   max(0, ceil((64p-14)/16), ceil((N-8-2(M-1-64p))/8)) <= i/8
     *   i/8 <= min(floor(j1/4), floor((2(N-1)-(M-1-j1))/16)).
     * Other groups are left untouched (about 70% of a 5:6 pair). Same size
     * and element placement as PARDTW_LAYOUT_PANEL; pardtw_dp treats the two
     * alike. */
    PARDTW_LAYOUT_PANEL_BAND = 2,
    /* The panel layout with only the 8-row groups that pardtw_subseq_dp reads:
     * the band of cells that can lie on a subsequence path (Sec. II-B), which
     * starts anywhere on row 0 and ends anywhere on row N-1. A group of panel
     * p is written when it holds a real cell that row 0 reaches (i <= 2j) and
     * a real cell that reaches row N-1 ((N-1-i) <= 2(M-1-j)); with
     * j1 = min(64p+63, M-1):
     *   max(0, ceil((N-8-2(M-1-64p))/8)) <= i/8 <= floor(j1/4).
     * Same size and element placement as PARDTW_LAYOUT_PANEL. */
    PARDTW_LAYOUT_PANEL_SUBSEQ_BAND = 3
} pardtw_layout;

#define PARDTW_PAIR_OK 0
#define PARDTW_PAIR_INFEASIBLE 1

/* Number of floats a cost buffer of the given layout occupies (0 on bad args). */
size_t pardtw_cost_elems(int64_t n, int64_t m, pardtw_layout layout);

/* Host-side helper: the 8-row groups [*lo, *hi] of column panel p (0 <= p <
 * ceil(M/64)) that PARDTW_LAYOUT_PANEL_BAND writes and pardtw_dp reads,
 * clamped to [0, ceil(N/8) - 1]; empty when *lo > *hi. Calls no HIP API.
 * PARDTW_ERR_INVALID_ARG on bad sizes, p out of range or null outputs. */
pardtw_status pardtw_band_groups(int64_t n, int64_t m, int64_t p, int64_t* lo, int64_t* hi);

/* Bytes of the backtrace buffer written by pardtw_dp (0 on bad args). Codes
 * use 64-column panels and 8-row groups with a column's 8 codes contiguous:
 *   byte((i,j)) = ((p*G + i/8)*64 + (j%64))*8 + i%8,  p = j/64, G = ceil(N/8).
 * pardtw_bp_unpack converts it to a plain row-major N x M int8 matrix. */
size_t pardtw_bp_bytes(int64_t n, int64_t m);

/* Bytes of device workspace pardtw_dp needs (0 on bad args). The workspace
 * carries boundary columns between column panels (16 B per row for at most
 * 257 boundaries in flight: 16 * N * min(ceil(M/64), 257) bytes, reused
 * round robin), a launch counter and, for the fused-cost DP, the inverse
 * norms of the rows of X. Zero it
 * once before its first use; afterwards it can be reused by any number of
 * pardtw_dp calls (of any size that fits) issued one after another on one
 * stream. Calls that overlap in time must not share a workspace. */
size_t pardtw_dp_workspace_bytes(int64_t n, int64_t m);

/* a1 + a2: pairwise cosine-distance matrix (Sec. IV) as an MFMA GEMM.
 *   X [device, n*d FP32], Y [device, m*d FP32]: row-major features.
 *   prec: PARDTW_PREC_F32 or PARDTW_PREC_BF16 (BF16 operands, FP32 accumulate;
 *         the norms are taken from the same BF16-rounded values).
 *   layout: PARDTW_LAYOUT_ROW, PARDTW_LAYOUT_PANEL or PARDTW_LAYOUT_PANEL_BAND.
 *   C [device, pardtw_cost_elems(n,m,layout) floats]: overwritten. A frame of
 *   zero norm is treated as the zero vector, so its cost is 1. */
pardtw_status pardtw_cost(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                          pardtw_prec prec, pardtw_layout layout, float* C, hipStream_t stream);

/* a3: the accumulated-cost dynamic program (Sec. II-D, Sec. III-B), swept as a
 * staircase wavefront: every 64-column panel advances one row per step and
 * each panel trails its left neighbour by a few rows, so all cells whose
 * predecessors are final are computed concurrently. Keeps only the last two
 * rows of D per panel on chip and writes one code byte per cell.
 *   C [device]: cost in the given layout (FP32; costs are not clamped). Only
 *   the band groups described at PARDTW_LAYOUT_PANEL_BAND are read.
 *   bp [device, pardtw_bp_bytes(n,m) bytes]: codes, layout as documented
 *   above: 0 = (1,1), 1 = (1,2), 2 = (2,1) for every cell that can lie on a
 *   path from (0,0) to (n-1,m-1) (reachable from the origin and able to reach
 *   the end), 3 at (0,0); the bytes of every other cell are unspecified.
 *   total [device, 1 float]: D[n-1, m-1] in FP32 (+inf if infeasible).
 *   pair_status [device, 1 int32]: PARDTW_PAIR_OK / PARDTW_PAIR_INFEASIBLE.
 *   workspace [device, >= pardtw_dp_workspace_bytes(n,m)], see above.
 * Per-cell arithmetic (fixed for bit-identical results across schedules):
 *   cand_r = fmaf(w_r, C[i,j], D_pred_r) in FP32; the winner is chosen by
 *   strict less-than in the order r = 0, 1, 2. */
pardtw_status pardtw_dp(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                        float* total, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* pardtw_dp with an explicit schedule: panels_per_workgroup in {1, 2, 4, 8}
 * consecutive 64-column panels share one workgroup (their boundary columns
 * pass through LDS); 0 picks it from the problem size. Every schedule gives
 * bit-identical results; the batched planner times them to choose. */
pardtw_status pardtw_dp_ex(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                           float* total, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                           int32_t panels_per_workgroup, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): pardtw_dp
 * with its workspace taken from a static device array of
 * PARDTW_NOALLOC_SCRATCH_BYTES bytes that the library holds on each GPU it
 * runs on until the process ends. Same arguments, results and per-cell
 * arithmetic as pardtw_dp, minus the workspace. It calls no allocating
 * routine; on its first call on a device it looks up the array's device
 * address (hipGetSymbolAddress) with that device current.
 *   PARDTW_ERR_WORKSPACE when pardtw_dp_workspace_bytes(n, m) exceeds
 *   PARDTW_NOALLOC_SCRATCH_BYTES (16 B per row of X for each of
 *   min(ceil(m/64), 257) record columns: about n*m <= 2.6e8 cells up to 16448
 *   columns, n <= 16300 beyond; 15000 x 15000 fits, 50000 x 60000 does not).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (boundary records tagged by a launch counter, so stale contents
 * are never mistaken for new ones): calls that overlap in time on one GPU,
 * from any stream or thread, race and must not be issued. */
#define PARDTW_NOALLOC_SCRATCH_BYTES (64u << 20)

pardtw_status pardtw_dp_noalloc(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                                float* total, int32_t* pair_status, hipStream_t stream);

/* The DP with the cost computed inside it, as ParDTW does (Sec. II-D): no cost
 * matrix is written or read, so the DP moves one byte per cell (its codes).
 * Each 64-column panel's costs are produced 16 rows at a time by a producer
 * wave running the cost GEMM's own MFMA slab into LDS, so every cost, code,
 * total and status is bit for bit that of pardtw_cost (FP32) followed by
 * pardtw_dp.
 *   X [device, n*d FP32], Y [device, m*d FP32]: row-major features, 1 <= d <= 16
 *   (PARDTW_ERR_UNSUPPORTED otherwise).
 *   bp, total, pair_status, workspace: as pardtw_dp.
 *   panels_per_workgroup: 0 (chosen from the size), 1, 2 or 4. */
pardtw_status pardtw_dp_fused(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, uint8_t* bp,
                              float* total, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                              int32_t panels_per_workgroup, hipStream_t stream);

/* a4: backtrace (Sec. II-D, Sec. VI-C) from (n-1, m-1) along the codes.
 *   bp [device]: codes written by pardtw_dp for the same (n, m).
 *   pair_status [device, 1 int32]: as written by pardtw_dp.
 *   path [device, 2*min(n,m) int32]: (i, j) pairs in forward order, from (0,0).
 *   path_len [device, 1 int32]: number of pairs written (0 if infeasible). */
pardtw_status pardtw_backtrace(const uint8_t* bp, int64_t n, int64_t m, const int32_t* pair_status,
                               int32_t* path, int32_t* path_len, hipStream_t stream);

/* a4, split walk: the path pardtw_backtrace returns, walked by many
 * workgroups. The rows are cut into S segments of R rows (R = max(512,
 * ceil(N/256))); each segment is walked from a guessed start (the diagonal,
 * clamped to the band), then again from where the segment above ended; one
 * workgroup then checks, from the last segment down, that every segment
 * started where the one above ended, and walks again serially any that did
 * not, so the result never depends on the guesses (Sec. VI-C puts the
 * backtrace on one thread; paths from nearby cells merge within a few dozen
 * steps, which is what makes the guesses pay).
 *   bp, n, m, pair_status, path, path_len: as for pardtw_backtrace.
 *   workspace [device, >= pardtw_backtrace_parallel_bytes(n, m) bytes,
 *     16-byte aligned]: segment starts, ends and cells (8 B per row); no
 *     initialisation needed. Calls that overlap in time must not share it.
 * Errors: PARDTW_ERR_INVALID_ARG (null or misaligned pointers, bad sizes),
 * PARDTW_ERR_WORKSPACE (workspace too small). Corrupt codes give path_len 0,
 * as in the serial walk. Five kernels on `stream`; pairs of at most 1024 rows
 * (two segments or fewer) take the one-workgroup walk instead. */
size_t pardtw_backtrace_parallel_bytes(int64_t n, int64_t m);
pardtw_status pardtw_backtrace_parallel(const uint8_t* bp, int64_t n, int64_t m, const int32_t* pair_status,
                                        int32_t* path, int32_t* path_len, void* workspace,
                                        size_t workspace_bytes, hipStream_t stream);

/* Inspection helper: the DP's backtrace buffer as a row-major n x m int8
 * matrix out [device, n*m bytes]. */
pardtw_status pardtw_bp_unpack(const uint8_t* bp, int64_t n, int64_t m, int8_t* out,
                               hipStream_t stream);

/* ---- Packed codes: 2 bits per cell (Sec. VI-D stores the transition types as
 * 2-bit values) -------------------------------------------------------------
 * A memory mode, not the throughput default: the codes take a quarter of the
 * bytes, so longer pairs fit (with the fused cost the DP then needs 0.25 B per
 * cell plus O(N) of workspace, against 1 B per cell for byte codes), at about
 * a tenth more sweep time. Layout: one 16-bit word per column and 8-row
 * group, row r of the group in bits 2r, 2r+1:
 *   word((i,j)) = (p*G + i/8)*64 + (j%64),  p = j/64, G = ceil(N/8),
 * the same codes as the byte layout (0, 1, 2 by step, 3 at the origin), on the
 * same band. pardtw_bp2_bytes gives the buffer size (0 on bad args). */
size_t pardtw_bp2_bytes(int64_t n, int64_t m);

/* pardtw_dp with packed codes: same arguments and results, bp2 [device,
 * pardtw_bp2_bytes(n,m) bytes, 16-byte aligned]. Layouts PANEL or PANEL_BAND
 * (PARDTW_ERR_UNSUPPORTED for ROW). */
pardtw_status pardtw_dp_packed(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint16_t* bp2,
                               float* total, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                               hipStream_t stream);

/* pardtw_dp_fused with packed codes (FP32 features, 1 <= d <= 16). */
pardtw_status pardtw_dp_fused_packed(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                     uint16_t* bp2, float* total, int32_t* pair_status, void* workspace,
                                     size_t workspace_bytes, hipStream_t stream);

/* pardtw_backtrace over packed codes: the same path. bp2 16-byte aligned. */
pardtw_status pardtw_backtrace_packed(const uint16_t* bp2, int64_t n, int64_t m, const int32_t* pair_status,
                                      int32_t* path, int32_t* path_len, hipStream_t stream);

/* pardtw_backtrace_parallel over packed codes (bp2 16-byte aligned); the same
 * path as pardtw_backtrace_packed. */
pardtw_status pardtw_backtrace_packed_parallel(const uint16_t* bp2, int64_t n, int64_t m,
                                               const int32_t* pair_status, int32_t* path, int32_t* path_len,
                                               void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Inspection helper: packed codes as a row-major n x m int8 matrix. */
pardtw_status pardtw_bp2_unpack(const uint16_t* bp2, int64_t n, int64_t m, int8_t* out, hipStream_t stream);

/* Checkpointed DTW: the exact path without the n x m code matrix, for pairs
 * whose codes would not fit in memory (Sec. II-D names memory as the limit on
 * length and cites a divide-and-conquer recomputation as the way past it).
 * Memory is 8 m / K bytes per row of X (checkpoints) instead of m (codes);
 * the recomputation adds about n K cells to the sweep's n m.
 *
 * pardtw_dp_fused_ckpt: the fused DP (pardtw_dp_fused's arithmetic, so the
 * same total and status bits) writing no codes; instead the FP32 D of rows
 * bK-2 and bK-1 for every b >= 1 with bK < n, each row over ceil(m/64)*64
 * columns (columns past m hold junk), into
 *   ckpt [device, >= pardtw_ckpt_bytes(n, m, K) bytes, 4-byte aligned],
 *   checkpoint row 2(b-1) = row bK-2, row 2(b-1)+1 = row bK-1.
 *   rows_per_block K: a multiple of 16 in [16, 256]
 *   (PARDTW_ERR_INVALID_ARG otherwise).
 *   X, Y, d, total, pair_status, workspace: as pardtw_dp_fused.
 * Only band cells of a checkpoint row (on some path from (0,0) to
 * (n-1,m-1)) are specified; other cells hold +inf or junk.
 * PARDTW_ERR_WORKSPACE if ckpt or workspace is missing or short.
 *
 * pardtw_ckpt_backtrace: the path, from pardtw_dp_fused_ckpt's checkpoints
 * with the same X, Y and K. One workgroup recomputes, block by block from the
 * last, the codes of the cells the path can reach in the block, with the
 * sweep's own instructions, and follows them: path and path_len are
 * identical to pardtw_dp_fused (or pardtw_cost + pardtw_dp) followed by
 * pardtw_backtrace.
 *   path [device, 2*min(n,m) int32], path_len [device, 1 int32]: as
 *   pardtw_backtrace (0 if pair_status is not PARDTW_PAIR_OK).
 * Both run on `stream` without host synchronisation or allocation. */
size_t pardtw_ckpt_bytes(int64_t n, int64_t m, int32_t rows_per_block);

pardtw_status pardtw_dp_fused_ckpt(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                   int32_t rows_per_block, float* ckpt, size_t ckpt_bytes, float* total,
                                   int32_t* pair_status, void* workspace, size_t workspace_bytes,
                                   hipStream_t stream);

pardtw_status pardtw_ckpt_backtrace(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                    int32_t rows_per_block, const float* ckpt, size_t ckpt_bytes,
                                    const int32_t* pair_status, int32_t* path, int32_t* path_len,
                                    hipStream_t stream);

/* pardtw_ckpt_backtrace's path from a split walk over runs of blocks (the
 * split walk of pardtw_backtrace_parallel: runs of R = K max(4, ceil(N / 256K))
 * rows, each walked block by block by its own workgroup from a guessed start,
 * then from where the run above ended, then checked from the last run down
 * with a serial rewalk of any run that started elsewhere). Same arguments,
 * plus workspace [device, >= pardtw_ckpt_backtrace_parallel_bytes(n, m,
 * rows_per_block) bytes, 16-byte aligned; no initialisation needed]. Pairs of
 * at most two runs take the one-workgroup walk. PARDTW_ERR_WORKSPACE if the
 * workspace is too small. */
size_t pardtw_ckpt_backtrace_parallel_bytes(int64_t n, int64_t m, int32_t rows_per_block);
pardtw_status pardtw_ckpt_backtrace_parallel(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                             int32_t rows_per_block, const float* ckpt, size_t ckpt_bytes,
                                             const int32_t* pair_status, int32_t* path, int32_t* path_len,
                                             void* workspace, size_t workspace_bytes, hipStream_t stream);

/* a6: gradient of g * J with the optimal path held fixed (the paper motivates
 * backpropagating through the optimal alignment path, Sec. I):
 *   J = sum over path cells (i,j) of w_ij * C[i,j], w = 1 at (0,0), else the
 *   weight of the step that lands on (i,j);
 *   dC/dx = -(v - <u,v> u)/|x|,  dC/dy = -(u - <u,v> v)/|y|,  u = x/|x|, v = y/|y|.
 *   X, Y [device FP32], path/path_len [device] from pardtw_backtrace,
 *   g_total [device, 1 float]: upstream gradient dL/dJ.
 *   dX [device, n*d FP32], dY [device, m*d FP32]: overwritten; rows and
 *   columns the path skips are zero, and an infeasible pair gives zeros. */
pardtw_status pardtw_path_grad(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                               const int32_t* path, const int32_t* path_len, const float* g_total,
                               float* dX, float* dY, hipStream_t stream);

/* Compensated total of a path: its cost (Sec. V: the start cell's cost plus,
 * per step, the step's weight times the cost of the cell it lands on) summed
 * in two-float arithmetic, each product and each addition's FP32 rounding
 * error carried exactly in a second float, and rounded once at the end. The
 * DP's own total rounds at every step, so on long paths it drifts (about
 * 1e-4 relative at 600000 x 600000); this one stays at the FP32 rounding of
 * the costs themselves. Costs are those of the FP32 features, the cosine
 * distance evaluated as |x/|x| - y/|y||^2 / 2 (equal to 1 - <x,y>/(|x||y|),
 * without its cancellation for nearly parallel frames; 1 for a zero frame).
 *   X [device, n*d FP32], Y [device, m*d FP32], path/path_len [device] as
 *   written by pardtw_backtrace or pardtw_ckpt_backtrace.
 *   total [device, 1 float]: the path's cost, +inf when path_len is 0.
 *   workspace [device, >= pardtw_path_total_bytes() bytes, 8-byte aligned]:
 *     the pieces' partial sums; no initialisation needed. Calls that overlap
 *     in time must not share it.
 * The path is cut into 256 contiguous pieces by its length alone, summed one
 * per workgroup and then added in a fixed tree, so the result does not depend
 * on the schedule. Two kernels on `stream`; no allocation or synchronisation.
 * PARDTW_ERR_WORKSPACE if the workspace is too small. */
size_t pardtw_path_total_bytes(void);
pardtw_status pardtw_path_total(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                const int32_t* path, const int32_t* path_len, float* total, void* workspace,
                                size_t workspace_bytes, hipStream_t stream);

/* ---- a5: batched form -----------------------------------------------------
 * Many independent pairs of uneven lengths aligned together (the problem of
 * Sec. III for each pair). A plan fixes the pair lengths: pair b has n_b rows
 * of X and m_b rows of Y, all with d features. Host data is read only during
 * pardtw_plan_create; the plan owns small device tables (pair descriptors,
 * work lists) and is the only object the library allocates.
 *
 * Packed buffers (device, caller-owned):
 *   X_packed: sum n_b rows of d FP32; pair b starts at row x_off[b], the
 *             exclusive prefix sum of n_b. Y_packed likewise with m_b.
 *   paths_packed: 2 * pardtw_plan_path_capacity int32, 8-byte aligned; pair b
 *             writes its (i, j) pairs in forward order from entry 2*p_off[b],
 *             p_off the exclusive prefix sum of min(n_b, m_b).
 *   totals (FP32), path_len and pair_status (int32): one entry per pair.
 *   workspace: pardtw_plan_workspace_bytes bytes, 256-byte aligned, zeroed
 *             once before first use (it holds the cost panels, the codes and
 *             the DP's boundary records of every pair).
 * An infeasible pair gets status PARDTW_PAIR_INFEASIBLE, total +inf and
 * path_len 0, and no work.
 *
 * pardtw_align_batch runs cost -> DP -> backtrace for the whole batch: the DP
 * of all pairs is one persistent launch over (pair, panel group) items. It
 * makes no allocation, copy or host synchronisation, so it can be captured in
 * a hipGraph. Calls sharing a workspace must not overlap in time. */
typedef struct pardtw_plan pardtw_plan;

pardtw_status pardtw_plan_create(int32_t batch, const int64_t* n_host, const int64_t* m_host,
                                 int64_t d, pardtw_prec prec, pardtw_plan** plan);

/* Plan flags. PARDTW_PLAN_FUSED_COST: the DP computes the costs itself, as
 * pardtw_dp_fused does (FP32, d <= 16, else PARDTW_ERR_UNSUPPORTED): the
 * workspace holds no cost matrix, only the row norms of X, and results are bit
 * for bit those of the unfused plan. Its schedules use 1, 2 or 4 panels per
 * workgroup. */
#define PARDTW_PLAN_FUSED_COST 1

/* pardtw_plan_create with flags. */
pardtw_status pardtw_plan_create_ex(int32_t batch, const int64_t* n_host, const int64_t* m_host, int64_t d,
                                    pardtw_prec prec, int32_t flags, pardtw_plan** plan);
size_t pardtw_plan_workspace_bytes(const pardtw_plan* plan);
int64_t pardtw_plan_path_capacity(const pardtw_plan* plan); /* sum of min(n_b, m_b) */
void pardtw_plan_destroy(pardtw_plan* plan);

pardtw_status pardtw_align_batch(const pardtw_plan* plan, const float* X_packed, const float* Y_packed,
                                 void* workspace, size_t workspace_bytes, float* totals,
                                 int32_t* paths_packed, int32_t* path_len, int32_t* pair_status,
                                 hipStream_t stream);

/* Schedules of the batched DP: panels per workgroup (1, 2, 4, 8), item order
 * (0 = breadth: group 0 of every pair by decreasing size, then group 1, ...;
 * 1 = depth: all groups of the largest pair first) and resident workgroups.
 * A Segmental DTW plan's staircase schedules use breadth order only (its
 * fragments differ in length by one row at most, so depth order would run
 * them one after another). With PARDTW_PLAN_FUSED_COST, FP32, d <= 16 and
 * fragments of at most 256 rows it also has the fragment sweep: panels per
 * workgroup 0, one workgroup per fragment (`workgroups` = nfrag) whose waves
 * take the fragment's panels in turn; `order` then gives those waves (1, 2
 * or 4). Every schedule computes bit-identical results; only the speed
 * differs. pardtw_plan_schedule describes schedule `index` (-1 = the selected
 * one). */
int32_t pardtw_plan_num_schedules(const pardtw_plan* plan);
pardtw_status pardtw_plan_schedule(const pardtw_plan* plan, int32_t index, int32_t* panels_per_workgroup,
                                   int32_t* order, int32_t* workgroups);
int32_t pardtw_plan_selected(const pardtw_plan* plan);
pardtw_status pardtw_plan_select(pardtw_plan* plan, int32_t index);

/* Autotuner: computes the batch's costs once, times the DP of every schedule
 * on them (one warm-up, then `reps` launches, HIP events on `stream`) and
 * selects the fastest; *best_ms (may be NULL) receives its time per launch.
 * Synchronises the stream, so it is not capturable; totals, codes and
 * statuses are left as written by the last schedule tried. */
pardtw_status pardtw_plan_autotune(pardtw_plan* plan, const float* X_packed, const float* Y_packed,
                                   void* workspace, size_t workspace_bytes, float* totals,
                                   int32_t* paths_packed, int32_t* path_len, int32_t* pair_status,
                                   int32_t reps, float* best_ms, hipStream_t stream);

/* Batched twin of pardtw_path_grad over the plan's pairs, reading the paths
 * written by pardtw_align_batch. g_totals: one FP32 per pair. dX_packed /
 * dY_packed: shaped like X_packed / Y_packed, overwritten (zeros for skipped
 * rows and infeasible pairs). */
pardtw_status pardtw_path_grad_batch(const pardtw_plan* plan, const float* X_packed,
                                     const float* Y_packed, const int32_t* paths_packed,
                                     const int32_t* path_len, const float* g_totals, float* dX_packed,
                                     float* dY_packed, hipStream_t stream);

/* ---- Subsequence DTW and Segmental DTW (Sec. II-B, II-C, III-A) ------------
 * The paper's other GPU algorithm. Sequence A (la x d) is cut into nfrag
 * fragments of nearly equal length, fragment f being rows
 * [floor(f la / nfrag), floor((f+1) la / nfrag)). Each fragment (the query,
 * rows i) is aligned with all of sequence B (the reference, lb x d, columns j)
 * by subsequence DTW: steps (1,1), (1,2), (2,1) with weights 1, 1, 2 on the
 * cell a step lands on, a free start anywhere on the first query row,
 *   D[0,j] = C[0,j],
 *   D[i,j] = min(D[i-1,j-1] + C, D[i-1,j-2] + C, D[i-2,j-1] + 2C),
 * codes 0/1/2 as for DTW (exact ties to the lowest), 3 on row 0. The score of
 * an end column is S[j] = D[n-1, j]; every such path weighs n, so scores of
 * different ends compare directly. A cell is reachable iff i <= 2j, so S[j] is
 * +inf for 2j < n-1. The fragments' scores stacked as rows give the
 * segment-level cost matrix S (nfrag x lb), and the fragment end columns
 * come from it:
 *   variant 0, NSDTW: each fragment ends at its lowest score (the first such
 *     column); total = the sum of those scores.
 *   variant 1, WSDTW: Dseg[f,j] = min(Dseg[f,j-1], Dseg[f-1,j-hop] + S[f,j])
 *     with Dseg[-1,.] = 0, Dseg[f,-1] = +inf, and +inf for f >= 1, j < hop; a
 *     match replaces the skip only when strictly smaller; total =
 *     Dseg[nfrag-1, lb-1]; ends are strictly increasing, at least hop apart.
 *     hop = max(1, floor(la / (2 nfrag))): the shortest stretch of B a fragment
 *     can match under a warping factor of at most 2.
 * Each fragment is then backtraced from its end to row 0, and the fragment
 * paths, shifted to A's row numbering and concatenated, are the alignment.
 * The scores and codes are exactly those of the whole-reference subsequence
 * DP, which is what the paper's overlapping reference chunks compute (Sec.
 * III-A); here the staircase sweep already keeps every panel of B busy, so no
 * chunk is recomputed. */
#define PARDTW_NSDTW 0
#define PARDTW_WSDTW 1

/* Host-side helper: the 8-row groups [*lo, *hi] of panel p that
 * PARDTW_LAYOUT_PANEL_SUBSEQ_BAND writes and pardtw_subseq_dp reads, clamped to
 * [0, ceil(N/8) - 1]; empty when *lo > *hi. Errors as pardtw_band_groups. */
pardtw_status pardtw_subseq_band_groups(int64_t n, int64_t m, int64_t p, int64_t* lo, int64_t* hi);

/* Subsequence DP of one fragment (n rows) against the reference (m columns),
 * swept as pardtw_dp sweeps DTW, with the same per-cell arithmetic:
 * cand_r = fmaf(w_r, C, D_pred_r), w = (1, 1, 2), strict less-than in order.
 *   C [device]: cost in layout ROW, PANEL or PANEL_SUBSEQ_BAND (for the last,
 *   only the groups it writes are read).
 *   bp [device, pardtw_bp_bytes(n,m)]: codes in the layout of pardtw_dp,
 *   defined on the subsequence band (3 on row 0); other bytes unspecified.
 *   scores [device, m floats]: S[j] = D[n-1, j] (+inf where unreachable).
 *   pair_status [device, 1 int32]: PARDTW_PAIR_OK, or PARDTW_PAIR_INFEASIBLE
 *   when no end is reachable (n-1 > 2(m-1); every score +inf, nothing swept).
 *   workspace [device, >= pardtw_dp_workspace_bytes(n,m)], as for pardtw_dp.
 * PARDTW_ERR_UNSUPPORTED for PARDTW_LAYOUT_PANEL_BAND. */
pardtw_status pardtw_subseq_dp(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                               float* scores, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                               hipStream_t stream);

/* pardtw_subseq_dp with the cost computed inside the DP, as pardtw_dp_fused:
 * scores and codes bit for bit those of pardtw_cost (FP32) + pardtw_subseq_dp.
 * 1 <= d <= 16. */
pardtw_status pardtw_subseq_dp_fused(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, uint8_t* bp,
                                     float* scores, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                                     hipStream_t stream);

/* Backtrace of a subsequence path from (n-1, *end_col) to row 0 along the
 * codes of pardtw_subseq_dp.
 *   end_col [device, 1 int32]: end column; a column outside [0, m) or one row
 *   n-1 cannot reach (2 end < n-1) gives path_len 0.
 *   path [device, 2*n int32, 8-byte aligned]: (i, j) pairs in forward order.
 *   path_len [device, 1 int32]: pairs written (0 when malformed codes stop
 *   the walk). */
pardtw_status pardtw_subseq_backtrace(const uint8_t* bp, int64_t n, int64_t m, const int32_t* end_col,
                                      int32_t* path, int32_t* path_len, hipStream_t stream);

/* Device workspace of pardtw_segment_ends (0 on bad args). Zero it once
 * before first use; calls sharing it must not overlap in time. */
size_t pardtw_segment_workspace_bytes(int64_t nfrag, int64_t m);

/* Segment level (Sec. II-C steps 3-4, or NSDTW's choice): fragment ends from
 * the stacked scores, as described above. The WSDTW program runs one
 * workgroup per fragment row, each scanning its row in tiles as soon as the
 * row before has published the tile it needs.
 *   scores [device, nfrag*m FP32, row-major]: S, row f = fragment f.
 *   hop >= 1; variant PARDTW_NSDTW or PARDTW_WSDTW.
 *   ends [device, nfrag int32]: end column per fragment (-1 when infeasible).
 *   total [device, 1 float]: the segment-level total in FP32 (+inf when no
 *   placement has a finite score).
 *   status [device, 1 int32]: PARDTW_PAIR_OK / PARDTW_PAIR_INFEASIBLE. */
pardtw_status pardtw_segment_ends(const float* scores, int64_t nfrag, int64_t m, int64_t hop, int32_t variant,
                                  void* workspace, size_t workspace_bytes, int32_t* ends, float* total,
                                  int32_t* status, hipStream_t stream);

/* A plan for Segmental DTW of A (la x d) against B (lb x d) with nfrag
 * fragments (1 <= nfrag <= la); flags as for pardtw_plan_create_ex (0 or
 * PARDTW_PLAN_FUSED_COST). It is a pardtw_plan: free it with
 * pardtw_plan_destroy, size its workspace (256-byte aligned, zeroed once) with
 * pardtw_plan_workspace_bytes, and choose its DP schedule with the schedule
 * calls above. */
pardtw_status pardtw_segplan_create(int64_t la, int64_t lb, int32_t nfrag, int64_t d, pardtw_prec prec,
                                    int32_t variant, int32_t flags, pardtw_plan** plan);

/* The autotuner of a Segmental DTW plan: computes the fragments' costs once,
 * times the subsequence DP under every schedule (one warm-up, then `reps`
 * launches) and selects the fastest; *best_ms (may be NULL) receives its time.
 * Synchronises the stream. */
pardtw_status pardtw_segplan_autotune(pardtw_plan* plan, const float* A, const float* B, void* workspace,
                                      size_t workspace_bytes, int32_t reps, float* best_ms, hipStream_t stream);

/* Byte offset, in the plan's workspace, of the stacked fragment scores S
 * (nfrag x lb FP32, row-major) left by the last pardtw_segmental_align call
 * (-1 for a plan of pairs). */
int64_t pardtw_segplan_scores_offset(const pardtw_plan* plan);

/* The segment hop of a Segmental DTW plan, max(1, floor(la / (2 nfrag))): the
 * column advance of a segment-level match (Sec. II-C), fixed at plan
 * creation. -1 for a plan of pairs or a null plan. */
int64_t pardtw_segplan_hop(const pardtw_plan* plan);

/* First row of A of fragment f, floor(f la / nfrag), for 0 <= f < nfrag
 * (Sec. II-B: fragments of approximately equal length); f = nfrag gives la.
 * -1 for f out of range, a plan of pairs or a null plan. */
int64_t pardtw_segplan_fragment_start(const pardtw_plan* plan, int32_t f);

/* Segmental DTW with one call: the cost GEMM of every fragment against B (only
 * the subsequence band), the subsequence DP of all fragments as one persistent
 * launch, the segment-level program, the fragments' backtraces (one workgroup
 * each, or the split walk of pardtw_backtrace_parallel for a fragment of more
 * than 1024 rows; the same paths) and their concatenation. No allocation, copy or synchronisation; it
 * can be captured in a hipGraph.
 *   A [device, la*d FP32], B [device, lb*d FP32].
 *   total [device, 1 float], ends [device, nfrag int32], status [device, 1
 *   int32]: as pardtw_segment_ends.
 *   path [device, 2*la int32, 8-byte aligned]: the concatenated alignment,
 *   (i, j) pairs with i in A's numbering, fragment by fragment (i strictly
 *   increases; j increases within a fragment).
 *   path_len [device, 1 int32]: pairs written (0 when infeasible). */
pardtw_status pardtw_segmental_align(const pardtw_plan* plan, const float* A, const float* B, void* workspace,
                                     size_t workspace_bytes, float* total, int32_t* ends, int32_t* path,
                                     int32_t* path_len, int32_t* status, hipStream_t stream);

const char* pardtw_status_string(pardtw_status status);

#ifdef __cplusplus
}
#endif

#endif /* PARDTW_H */
