// Internal definitions of the batched form: the per-pair descriptor that the
// plan keeps in device memory and the batch launchers of each kernel.
#pragma once

#include "common.h"

namespace pardtw {

// One pair of a batch. Offsets are element offsets from the caller's packed
// features (rows), the plan's workspace regions (floats / bytes / records) and
// the packed path buffer (int32 pairs).
struct BatchPair {
    int64_t n, m;
    int64_t x_off, y_off;  // first row of the pair in X_packed / Y_packed
    int64_t c_off;         // first float of the pair's cost panels
    int64_t bp_off;        // first byte of the pair's codes
    int64_t rec_off;       // first boundary record (uint64) of the pair
    int64_t path_off;      // first (i, j) entry of the pair's path
    int64_t G;             // 8-row groups
    int64_t tile0;         // first cost workgroup of the pair in the batch numbering
    int64_t rx_off;        // fused cost: first float of the pair's row-norm area
    int32_t P;             // column panels
    int32_t feasible;      // some path exists (to (n-1, m-1), or to row n-1 for a fragment)
    int32_t band;          // cost groups written: 1 the DTW path band, 2 the subsequence band
    int32_t split;         // 1: backtrace by the split walk (a SegPair lists it), 0: one workgroup
};

// A pair of a batch whose backtrace is the split walk of
// pardtw_backtrace_parallel: its segments, and where their state lives in the
// plan's split region (segment records, then cells).
struct SegPair {
    int32_t pair;       // index in the batch
    int32_t R, S;       // rows per segment, segments
    int32_t seg0;       // first segment in the batch numbering
    int64_t info_off;   // first of its 2 S segment records
    int64_t cells_off;  // first int32 of its S R cell pairs
};

// Work item of the persistent batched DP: panel group q of pair b.
struct DpItem {
    int32_t pair;
    int32_t group;
};

// Workgroups of the cost kernel for one (n, m) pair (panels x row-tile blocks).
int64_t cost_blocks(int64_t n, int64_t m);

pardtw_status cost_batch_launch(const BatchPair* pairs, const int32_t* tile_pair, int64_t tiles, const float* X,
                                const float* Y, int64_t d, pardtw_prec prec, float* Cbase, hipStream_t stream);

// Sweeps every item with one persistent launch; hdr/rec as in the single-pair
// DP (one header for the batch, records at each pair's rec_off).
// With `sub` every pair is a fragment of Segmental DTW: the subsequence DP,
// whose scores go to totals + b * m (fragments share m). With X (not null) the
// costs are computed inside the DP from X_packed, Y_packed (fused form): FP32
// with d <= 16 and the row norms at rxs (nw <= 4), or with `bf16` from BF16
// operands with d <= 128, d % 8 == 0 (nw <= 2); otherwise they are read from
// Cbase.
pardtw_status dp_batch_launch(const BatchPair* pairs, const DpItem* items, int32_t nitems, int nw, int grid,
                              const float* Cbase, const float* X, const float* Y, int64_t d, const float* rxs,
                              bool bf16, uint8_t* bpbase, float* totals, int32_t* status, void* dp_ws, bool sub,
                              hipStream_t stream);

// Segmental DTW fragments of at most frag_sweep_max_rows() rows (fused FP32
// costs, d <= 16): one workgroup per fragment sweeps all of its panels, its
// `waves` waves (1, 2 or 4) taking them in turn, with the batched DP's
// arithmetic (the same scores, codes and statuses).
int64_t frag_sweep_max_rows();
pardtw_status frag_sweep_launch(const BatchPair* pairs, int32_t nfrag, int64_t max_n, int waves, const float* X,
                                const float* Y, int64_t d, const float* rxs, uint8_t* bpbase, float* totals,
                                int32_t* status, hipStream_t stream);

// Row norms of every feasible pair for the fused batched DP (rx_floats(n_b)
// floats at rx_off each); max_n is the largest n_b.
pardtw_status row_norms_batch_launch(const BatchPair* pairs, int32_t batch, int64_t max_n, const float* X,
                                     int64_t d, float* rxs, hipStream_t stream);

pardtw_status backtrace_batch_launch(const BatchPair* pairs, int32_t batch, const uint8_t* bpbase,
                                     const int32_t* status, int32_t* paths, int32_t* path_len, hipStream_t stream);

// Segments of the split walk for a pair of n rows: R rows each, S of them; a
// pair is split when S > 2.
void split_shape(int64_t n, int& R, int& S);
size_t split_record_bytes();  // one segment record
// The split pairs' walks (nseg segments over nsplit pairs; seg_map[g] is the
// SegPair of segment g). Pairs with split == 0 are left to backtrace_batch_launch
// (DTW pairs, `ends` null, walked when status[pair] is OK) or to
// subseq_backtrace_batch_launch (Segmental DTW fragments, walked from ends[pair]).
pardtw_status split_backtrace_batch_launch(const BatchPair* pairs, const SegPair* sp, int32_t nsplit,
                                           const int32_t* seg_map, int32_t nseg, const uint8_t* bpbase,
                                           const int32_t* status, const int32_t* ends, void* records,
                                           int32_t* cells, int32_t* paths, int32_t* path_len, hipStream_t stream);

pardtw_status grad_batch_launch(const BatchPair* pairs, int32_t batch, int64_t max_cap, int64_t d, const float* X,
                                const float* Y, const int32_t* paths, const int32_t* path_len, const float* g,
                                float* dX, int64_t dX_count, float* dY, int64_t dY_count, hipStream_t stream);

// Fragment b walked from ends[b] to row 0 into its slot of n_b pairs at path_off
// (fragments with split set are left to split_backtrace_batch_launch).
pardtw_status subseq_backtrace_batch_launch(const BatchPair* pairs, int32_t batch, const uint8_t* bpbase,
                                            const int32_t* ends, int32_t* paths, int32_t* path_len,
                                            hipStream_t stream);

// Segment level of Segmental DTW (segment.hip).
size_t segment_workspace_bytes_impl(int64_t nf, int64_t m);
pardtw_status segment_ends_launch(const float* S, int64_t nf, int64_t m, int64_t hop, int variant, void* ws,
                                  int32_t* ends, float* total, int32_t* status, hipStream_t stream);
pardtw_status segment_gather_launch(const BatchPair* pairs, int32_t nf, const int32_t* slots,
                                    const int32_t* frag_len, const int32_t* status, int32_t* path,
                                    int32_t* path_len, hipStream_t stream);
pardtw_status segment_init_launch(const BatchPair* pairs, int32_t nf, float* scores, int32_t* frag_status,
                                  hipStream_t stream);

size_t dp_header_bytes();
size_t dp_record_bytes(int64_t n, int64_t m);  // boundary records of one pair

}  // namespace pardtw
