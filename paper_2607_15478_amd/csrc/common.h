// Internal definitions shared by the libpardtw HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pardtw.h"

namespace pardtw {

constexpr int kLanes = 64;        // wavefront width on CDNA4; one lane per column
constexpr int kPanel = 64;        // columns per panel (= kLanes)
constexpr int kBpRows = 8;        // rows per packed backtrace group (8 code bytes per lane)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t num_panels(int64_t m) { return ceil_div(m, kPanel); }
__host__ __device__ inline int64_t bp_groups(int64_t n) { return ceil_div(n, kBpRows); }

// Byte offset of cell (i, j) inside the backtrace buffer.
__host__ __device__ inline int64_t bp_offset(int64_t n, int64_t i, int64_t j) {
    const int64_t p = j / kPanel;
    return ((p * bp_groups(n) + i / kBpRows) * kLanes + (j % kPanel)) * kBpRows + (i % kBpRows);
}

// Sizes must stay representable: cells counted in int64, coordinates in int32.
inline bool valid_sizes(int64_t n, int64_t m) {
    return n > 0 && m > 0 && n < (int64_t(1) << 31) && m < (int64_t(1) << 31) &&
           n <= (int64_t(1) << 62) / m;
}

// Cells on some path from (0,0) to (n-1,m-1) with the steps (1,1), (1,2),
// (2,1) (Sec. V): reachable from the origin, j <= 2i and i <= 2j, and able to
// reach the end, (m-1-j) <= 2(n-1-i) and (n-1-i) <= 2(m-1-j). Only they can lie
// on the optimal path. For column panel p (columns 64p .. 64p+63) the 8-row
// groups k that hold a cell of the first cone and a cell of the second (real
// cells only, i < n, j < m) are band_group_lo(p) .. band_group_hi(p), empty
// when lo > hi. Each bound follows from testing the cone against the group's
// box: a box [a1, a2] x [b1, b2] meets {j <= 2i, i <= 2j} iff b1 <= 2 a2 and
// a1 <= 2 b2.
__host__ __device__ inline int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

__host__ __device__ inline int64_t band_group_lo(int64_t p, int64_t n, int64_t m) {
    const int64_t j0 = p * kPanel;
    // origin cone: 64p <= 2(8k+7), and the panel must start within 2(n-1)
    int64_t lo = -floor_div(-(j0 - 14), 16);  // ceil((64p - 14) / 16)
    if (j0 > 2 * (n - 1)) return int64_t(1) << 40;
    // end cone: n-1-(8k+7) <= 2(m-1-64p)
    const int64_t le = -floor_div(-(n - 8 - 2 * (m - 1 - j0)), 8);
    if (le > lo) lo = le;
    return lo < 0 ? 0 : lo;
}

__host__ __device__ inline int64_t band_group_hi(int64_t p, int64_t n, int64_t m) {
    const int64_t j0 = p * kPanel;
    const int64_t j1 = j0 + kPanel - 1 < m - 1 ? j0 + kPanel - 1 : m - 1;  // last real column
    // origin cone: 8k <= 2 j1
    int64_t hi = floor_div(j1, 4);
    // end cone: m-1-j1 <= 2(n-1-8k)
    const int64_t he = floor_div(2 * (n - 1) - (m - 1 - j1), 16);
    if (he < hi) hi = he;
    return hi;
}

inline bool pair_feasible(int64_t n, int64_t m) {
    return (m - 1) <= 2 * (n - 1) && (n - 1) <= 2 * (m - 1);
}

// Subsequence DTW (Sec. II-B): a path starts anywhere on row 0 and ends
// anywhere on row n-1. A cell lies on one iff row 0 reaches it, i <= 2j, and
// it reaches row n-1 inside the matrix, (n-1-i) <= 2(m-1-j). Per column panel
// the 8-row groups holding a cell of each are sub_group_lo .. sub_group_hi
// (the same box tests as above).
__host__ __device__ inline int64_t sub_group_lo(int64_t p, int64_t n, int64_t m) {
    const int64_t le = -floor_div(-(n - 8 - 2 * (m - 1 - p * kPanel)), 8);
    return le < 0 ? 0 : le;
}

__host__ __device__ inline int64_t sub_group_hi(int64_t p, int64_t n, int64_t m) {
    const int64_t j1 = p * kPanel + kPanel - 1 < m - 1 ? p * kPanel + kPanel - 1 : m - 1;
    return floor_div(j1, 4);
}

// Floats of the fused DP's row-norm area for n rows: its producers' loop,
// padded to a multiple of three 16-row slabs, reads up to two slabs past its
// end; rows past n hold zeros.
__host__ __device__ inline int64_t rx_floats(int64_t n) { return (ceil_div(bp_groups(n), 2) + 5) * 16; }

// Checkpointed backtrace with blocks of K rows: D of rows bK-2 and bK-1 for
// every block b > 0, each row over all panel columns.
__host__ __device__ inline int64_t ckpt_count(int64_t n, int64_t K) { return (n - 1) / K; }
__host__ __device__ inline int64_t ckpt_floats(int64_t n, int64_t m, int64_t K) {
    return 2 * ckpt_count(n, K) * num_panels(m) * kPanel;
}
constexpr int kCkMaxRows = 256;  // the largest block the backtrace's window holds in LDS

// Some end column of row n-1 is reachable from row 0.
inline bool subseq_feasible(int64_t n, int64_t m) { return n - 1 <= 2 * (m - 1); }

// Device workspace header of the DP (followed by boundary records).
struct DpWsHeader {
    uint32_t epoch;    // launch counter; boundary records carry it as a tag
    uint32_t ticket;   // work-queue head for the persistent DP
    uint32_t pad[62];
    uint64_t sink[64]; // target of the DP's stores for chunks past the end
};
static_assert(sizeof(DpWsHeader) == 768, "header keeps records 256-byte aligned");

#define PARDTW_HIP_TRY(expr)                                  \
    do {                                                      \
        if ((expr) != hipSuccess) return PARDTW_ERR_HIP;      \
    } while (0)

inline pardtw_status launch_status() {
    return hipGetLastError() == hipSuccess ? PARDTW_OK : PARDTW_ERR_HIP;
}

}  // namespace pardtw
