// Lane-parallel tracing of a path through 32 rows of 2-bit codes, shared by
// the backtraces. Lane b of a wave holds column j - b of a window whose
// first row is the current row i; codes are 0 = (1,1), 1 = (1,2), 2 = (2,1),
// 3 = origin, and a step from column j - b moves to column j - b - 1 - (code
// & 1), so each step moves the path one or two lanes to the right.
#pragma once

#include "common.h"

namespace pardtw {
namespace {

// lane l receives lane l-1's value (lane 0 receives 0)
__device__ inline uint32_t from_prev_lane(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}

// Bits 0, 2, 4, ... of x to bits 0, 1, 2, ... (16 bits).
__device__ inline uint32_t even_bits(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    return (x | (x >> 8)) & 0x0000FFFFu;
}

// Row masks of one lane's window, bit 31 - a for row a: the code's bit 0 (the
// step takes two columns) and bit 1 (two rows).
struct WindowMasks {
    uint32_t two_cols, two_rows;
};

__device__ inline WindowMasks window_masks(uint32_t packed0, uint32_t packed1) {
    // row a of a half sits at bits 30-2a (low code bit), which even_bits moves to 15 - a
    WindowMasks w;
    w.two_cols = (even_bits(packed0) << 16) | even_bits(packed1);
    w.two_rows = (even_bits(packed0 >> 1) << 16) | even_bits(packed1 >> 1);
    return w;
}

// Traces the path through the window from lane 0, row 0 and returns each
// lane's path cell as a mask (bit 31 - a for row a; at most one bit). A step
// from row a of lane b goes to lane b + 1 + (code & 1), row a + 1 + (code >> 1);
// the frontier is empty once the path has left the 32 rows. Code 3 stops it,
// and so does a row outside `live` (bit 31 - a for row a): the cell the path
// enters there is still marked.
__device__ inline uint32_t trace_window_live(const WindowMasks& w, uint32_t live, int lane) {
    const uint32_t diag = (~(w.two_cols | w.two_rows) & live) >> 1;     // code 0: next lane, next row
    const uint32_t down = ((w.two_rows & ~w.two_cols) & live) >> 2;     // code 2: next lane, two rows on
    const uint32_t over = ((w.two_cols & ~w.two_rows) & live) >> 1;     // code 1: two lanes on, next row
    uint32_t f = lane == 0 ? 0x80000000u : 0u;
    uint32_t on = f;
    for (int t = 0; t < 32; t += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint32_t f1 = f >> 1, f2 = f >> 2;
            const uint32_t hop = from_prev_lane(f1 & over);
            f = from_prev_lane((f1 & diag) | (f2 & down) | hop);
            on |= f;
        }
        if (__builtin_amdgcn_ballot_w64(f != 0) == 0) break;
    }
    return on;
}

__device__ inline uint32_t trace_window(const WindowMasks& w, int lane) { return trace_window_live(w, ~0u, lane); }

}  // namespace
}  // namespace pardtw
