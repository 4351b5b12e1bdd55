// The DP's row step (Sec. V: steps {(1,1),(1,2),(2,1)}, weights {2,3,3}; with
// SUB the subsequence weights {1,1,2}) on one wave that owns a 64-column
// panel, lane = column, and the LDS helpers its waves synchronise with. The
// full sweep and the checkpointed backtrace's window recomputation run these
// same instructions, so they produce the same bits.
#pragma once

#include "cost_slab.h"

namespace pardtw {
namespace {

constexpr int kChunk = kBpRows;  // rows per synchronisation chunk (= packed group)

__device__ inline int lds_get(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_put(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// LDS operations of one wave are performed in issue order; this only stops the
// compiler from moving memory accesses across the point.
__device__ inline void compiler_order() { asm volatile("" ::: "memory"); }

// lane l receives lane l-1's value; lane 0 receives `edge`.
__device__ inline float shift_in(float v, float edge) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v),
                                                      0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}

// One 8-row chunk of a panel. `lv0/lv1` hold the left boundary columns
// D[i0+r][64p-2] / D[i0+r][64p-1]; e0/e1 the same for row i0-1. The codes of
// the 8 rows come back one byte per row (row r in byte r of lo, hi), or with
// PACK as 2 bits per row in lo (row r in bits 2r, 2r+1; hi = 0).
template <bool SUB, bool PACK = false>
__device__ __attribute__((always_inline)) inline void dp_rows(const float (&cb)[kChunk], const float (&lv0)[kChunk],
                                                              const float (&lv1)[kChunk], float e0, float e1,
                                                              float& d1, float& s1p, uint32_t& lo, uint32_t& hi,
                                                              float (&best_r)[kChunk]) {
    lo = 0;
    hi = 0;
#pragma unroll
    for (int r = 0; r < kChunk; ++r) {
        const float c = cb[r];
        const float s1 = shift_in(d1, r == 0 ? e1 : lv1[r - 1]);  // D[i-1][j-1]
        const float s2 = shift_in(s1, r == 0 ? e0 : lv0[r - 1]);  // D[i-1][j-2]
        const float c0 = __builtin_fmaf(SUB ? 1.0f : 2.0f, c, s1);
        const float c1 = __builtin_fmaf(SUB ? 1.0f : 3.0f, c, s2);
        const float c2 = __builtin_fmaf(SUB ? 2.0f : 3.0f, c, s1p);
        const float best = __builtin_fminf(__builtin_fminf(c0, c1), c2);
        uint32_t code = (c1 == best) ? 1u : 2u;
        code = (c0 == best) ? 0u : code;
        // packed: 2 bits per row, rows 4-7 gathered apart and joined after
        // the loop, which keeps the OR chains short enough for the compiler
        // to interleave the code selection with the row arithmetic
        if (PACK) {
            if (r < 4) lo |= code << (2 * r);
            else hi |= code << (2 * r);
        } else if (r < 4) lo |= code << (8 * r);
        else hi |= code << (8 * (r - 4));
        d1 = best;
        s1p = s1;
        best_r[r] = best;
    }
    if (PACK) {
        lo |= hi;
        hi = 0;
    }
}

}  // namespace
}  // namespace pardtw
