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

// Cells reachable from (0,0) by the steps (1,1), (1,2), (2,1) are exactly those
// with j <= 2i and i <= 2j. For column panel p (columns 64p .. 64p+63), the
// 8-row groups that hold at least one such cell are reach_group_lo(p) ..
// reach_group_hi(p) (not clamped to the number of groups): group k is reached
// when 64p <= 2(8k+7) and 8k <= 2(64p+63).
__host__ __device__ inline int64_t reach_group_lo(int64_t p) {
    const int64_t jlo = p * kPanel;
    return jlo <= 14 ? 0 : (jlo - 14 + 15) / 16;
}
__host__ __device__ inline int64_t reach_group_hi(int64_t p) { return (p * kPanel + kPanel - 1) / 4; }

inline bool pair_feasible(int64_t n, int64_t m) {
    return (m - 1) <= 2 * (n - 1) && (n - 1) <= 2 * (m - 1);
}

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
