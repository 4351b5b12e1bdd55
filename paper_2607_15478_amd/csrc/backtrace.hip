// a4: backtrace of the optimal path (Sec. II-D keeps the full backtrace
// matrix; the path is recovered from (N-1, M-1) once the sweep is done).
//
// The walk is inherently serial. One wavefront walks it; the codes it needs
// are staged through LDS in windows of two adjacent 64-column panels x 64 rows
// (8 KB, read as contiguous 512-byte row groups of the DP's backtrace layout),
// since every step moves 1-2 rows and 1-2 columns up-left and so stays inside
// the current window for at least 32 steps.
#include "common.h"

namespace pardtw {
namespace {

constexpr int kWinGroups = 8;  // 8 groups of 8 rows = 64 rows per window

__global__ __launch_bounds__(64) void backtrace_kernel(const uint2* __restrict__ bp, int64_t n, int64_t m,
                                                       const int32_t* __restrict__ status, int32_t* path,
                                                       int32_t* path_len) {
    __shared__ uint2 win[2][kWinGroups][kLanes];
    __shared__ int64_t st[3];  // i, j, steps written
    const int lane = threadIdx.x;
    const int64_t cap = n < m ? n : m;
    if (*status != PARDTW_PAIR_OK) {
        if (lane == 0) *path_len = 0;
        return;
    }
    const int64_t G = bp_groups(n);
    int64_t i = n - 1, j = m - 1, len = 0;
    bool done = false;
    while (!done) {
        const int64_t pa = j / kPanel;
        const int64_t ghi = i / kBpRows;
        const int64_t g0 = ghi >= kWinGroups - 1 ? ghi - (kWinGroups - 1) : 0;
        for (int pp = 0; pp < 2; ++pp) {
            const int64_t pan = pa - pp;
            if (pan < 0) break;
            for (int gg = 0; gg < kWinGroups; ++gg) {
                const int64_t g = g0 + gg;
                if (g >= G) break;
                win[pp][gg][lane] = bp[(pan * G + g) * kLanes + lane];
            }
        }
        __syncthreads();
        if (lane == 0) {
            const int64_t rlo = g0 * kBpRows;
            const int64_t clo = (pa > 0 ? pa - 1 : 0) * kPanel;
            for (;;) {
                // record (i, j) at the back of the buffer; reversed at the end
                const int64_t pos = cap - 1 - len;
                path[2 * pos] = int32_t(i);
                path[2 * pos + 1] = int32_t(j);
                ++len;
                if (i == 0 && j == 0) { done = true; break; }
                const int pp = int(pa - j / kPanel);
                const uint2 w = win[pp][(i / kBpRows) - g0][j % kPanel];
                const int t = int(i % kBpRows);
                const uint32_t word = t < 4 ? w.x : w.y;
                const uint32_t code = (word >> (8 * (t & 3))) & 0xffu;
                if (code > 2 || len >= cap) { len = 0; done = true; break; }  // corrupt input: no path
                i -= (code == 2) ? 2 : 1;
                j -= (code == 1) ? 2 : 1;
                if (i < rlo || j < clo) break;
            }
            st[0] = i; st[1] = j; st[2] = len + (done ? (int64_t(1) << 40) : 0);
        }
        __syncthreads();
        i = st[0];
        j = st[1];
        len = st[2] & ((int64_t(1) << 40) - 1);
        done = (st[2] >> 40) != 0;
        __syncthreads();
    }
    // The walk filled [cap-len, cap) from the back, so the buffer already holds
    // the path in forward order there: shift it down to start at entry 0.
    const int64_t base = cap - len;
    __threadfence();
    __syncthreads();
    if (base > 0) {
        for (int64_t q0 = 0; q0 < len; q0 += kLanes) {
            const int64_t q = q0 + lane;
            int32_t v0 = 0, v1 = 0;
            if (q < len) { v0 = path[2 * (base + q)]; v1 = path[2 * (base + q) + 1]; }
            __syncthreads();
            if (q < len) { path[2 * q] = v0; path[2 * q + 1] = v1; }
            __syncthreads();
        }
    }
    if (lane == 0) *path_len = int32_t(len);
}

__global__ void bp_unpack_kernel(const uint8_t* __restrict__ bp, int64_t n, int64_t m, int8_t* __restrict__ out) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t i = idx / m, j = idx % m;
    out[idx] = int8_t(bp[bp_offset(n, i, j)]);
}

}  // namespace
}  // namespace pardtw

extern "C" pardtw_status pardtw_backtrace(const uint8_t* bp, int64_t n, int64_t m, const int32_t* pair_status,
                                          int32_t* path, int32_t* path_len, hipStream_t stream) {
    if (!bp || !pair_status || !path || !path_len || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    pardtw::backtrace_kernel<<<1, 64, 0, stream>>>(reinterpret_cast<const uint2*>(bp), n, m, pair_status, path,
                                                   path_len);
    return pardtw::launch_status();
}

extern "C" pardtw_status pardtw_bp_unpack(const uint8_t* bp, int64_t n, int64_t m, int8_t* out, hipStream_t stream) {
    if (!bp || !out || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    const int64_t cells = n * m;
    const int64_t blocks = pardtw::ceil_div(cells, 256);
    if (blocks > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    pardtw::bp_unpack_kernel<<<unsigned(blocks), 256, 0, stream>>>(bp, n, m, out);
    return pardtw::launch_status();
}
