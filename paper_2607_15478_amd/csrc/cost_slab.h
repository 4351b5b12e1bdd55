// The cosine cost (Sec. IV) of one 16-row x 64-column slab of a column panel,
// computed by one wave with MFMA: the unit shared by the cost GEMM, which
// stores slabs to HBM, and the fused DP, whose producer waves hand them to
// the DP waves through LDS. Both run these same instructions, so the fused DP
// sees bit for bit the costs the GEMM would have written.
//
//   C[i,j] = 1 - (<x_i, y_j> * rx_i) * ry_j,   rx_i = 1/|x_i| (0 for a zero frame)
//
// Lane layout (v_mfma_f32_16x16x4_f32, four 16x16 column blocks b): the lane
// holds rows row0 + 4*(lane/16) + r, r = 0..3, of column b*16 + lane%16, i.e.
// one 16-byte group-half per block in the panel layout (rows 0-3 or 4-7 of an
// 8-row group, one column).
#pragma once

#include "common.h"

namespace pardtw {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline float sum_groups(float v) {
    // lanes l, l^16, l^32, l^48 hold the four quarters of one row / column
    v += __shfl_xor(v, 16, 64);
    return v + __shfl_xor(v, 32, 64);
}

__device__ inline float inv_from_sq(float s) { return s > 0.0f ? 1.0f / __builtin_sqrtf(s) : 0.0f; }

// Final costs from the MFMA accumulators: rxl is the inverse norm of row
// lane%16 of the slab, ry[b] that of column b*16 + lane%16.
__device__ __attribute__((always_inline)) inline void costs_from_acc(const f32x4 (&acc)[4], float rxl,
                                                                     const float (&ry)[4], f32x4 (&v)[4]) {
    const int lane = threadIdx.x & 63;
    const int tr0 = 4 * (lane >> 4);
    float rx[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rx[r] = __shfl(rxl, tr0 + r, 64);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[b][r] = 1.0f - (acc[b][r] * rx[r]) * ry[b];
}

// FP32, d <= 16: feature k = 4t + g (g = lane/16) at MFMA step t. The column
// operands of panel p and their inverse norms, kept in registers while the
// panel's slabs are computed (zeros past m and past d).
__device__ __attribute__((always_inline)) inline void panel_operands_f32_small(const float* __restrict__ Y,
                                                                               int64_t m, int64_t d, int64_t p,
                                                                               float (&bv)[4][4], float (&ry)[4]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t col = p * kPanel + b * 16 + (lane & 15);
        float sq = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t k = 4 * t + g;
            bv[b][t] = (col < m && k < d) ? Y[col * d + k] : 0.0f;
            sq = __builtin_fmaf(bv[b][t], bv[b][t], sq);
        }
        ry[b] = inv_from_sq(sum_groups(sq));
    }
}

// The row operands of the slab of rows row0 .. row0+15 (zeros past n and d).
__device__ __attribute__((always_inline)) inline void slab_rows_f32_small(const float* __restrict__ X, int64_t n,
                                                                          int64_t d, int64_t row0, float (&av)[4]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int64_t arow = row0 + (lane & 15);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t k = 4 * t + g;
        av[t] = (arow < n && k < d) ? X[arow * d + k] : 0.0f;
    }
}

// The same operands for loads issued ahead of use: every lane loads, from the
// feature or from `zeros` (at least 16 zero floats) past n and d, so no load
// sits under a branch and the compiler's count of loads in flight stays exact.
__device__ __attribute__((always_inline)) inline void slab_rows_f32_small_ahead(const float* __restrict__ X,
                                                                                const float* __restrict__ zeros,
                                                                                int64_t n, int64_t d, int64_t row0,
                                                                                float (&av)[4]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int64_t arow = row0 + (lane & 15);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t k = 4 * t + g;
        const float* src = (arow < n && k < d) ? X + arow * d + k : zeros + k;
        av[t] = *src;
    }
}

// MFMA steps over features 4t + g, d <= 16. Step t is issued only when
// 4t < d: past d both operands are zero, so a skipped step would only have
// added zeros (at most turning a -0 or denormal sum into +0, which gives the
// same cost 1 - (acc rx) ry), and the costs are the same bits (d = 12 takes
// three steps, not four). Pass 16 to run every step.
__device__ __attribute__((always_inline)) inline void slab_acc_f32_small(int64_t d, const float (&av)[4],
                                                                         const float (&bv)[4][4], f32x4 (&acc)[4]) {
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (4 * t < d)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], bv[b][t], acc[b], 0, 0, 0);
}

// The slab's costs from its row operands and the panel operands.
__device__ __attribute__((always_inline)) inline void slab_costs_from_rows(int64_t d, const float (&av)[4],
                                                                           const float (&bv)[4][4],
                                                                           const float (&ry)[4], f32x4 (&v)[4]) {
    float sa = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) sa = __builtin_fmaf(av[t], av[t], sa);
    f32x4 acc[4];
    slab_acc_f32_small(d, av, bv, acc);
    costs_from_acc(acc, inv_from_sq(sum_groups(sa)), ry, v);
}

// The slab of rows row0 .. row0+15 against the panel operands.
__device__ __attribute__((always_inline)) inline void slab_costs_f32_small(const float* __restrict__ X, int64_t n,
                                                                           int64_t d, int64_t row0,
                                                                           const float (&bv)[4][4],
                                                                           const float (&ry)[4], f32x4 (&v)[4]) {
    float av[4];
    slab_rows_f32_small(X, n, d, row0, av);
    slab_costs_from_rows(d, av, bv, ry, v);
}

// The inverse norm of row i (d <= 16) as the slab computes it: lane group g
// sums the squares of features 4t + g over t, and sum_groups adds the four
// partial sums as (s0 + s1) + (s2 + s3) (the same bits on every lane, since
// each addition is commutative). 0 past n.
// The same from the row's 16 features (zeros past d): an all-zero row gives 0.
__device__ inline float inv_norm16(const float (&x)[16]) {
    float sg[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) s = __builtin_fmaf(x[4 * t + g], x[4 * t + g], s);
        sg[g] = s;
    }
    return inv_from_sq((sg[0] + sg[1]) + (sg[2] + sg[3]));
}

__device__ inline float row_inv_norm_f32_small(const float* __restrict__ X, int64_t n, int64_t d, int64_t i) {
    if (i >= n) return 0.0f;
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = k < d ? X[i * d + k] : 0.0f;
    return inv_norm16(x);
}

// Costs of a slab from its accumulators, with the row inverse norms of the
// lane's rows given (rx4[r] for row 4*(lane/16) + r).
__device__ __attribute__((always_inline)) inline void costs_from_acc_rx(const f32x4 (&acc)[4], const f32x4& rx4,
                                                                        const float (&ry)[4], f32x4 (&v)[4]) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[b][r] = 1.0f - (acc[b][r] * rx4[r]) * ry[b];
}

// ---- BF16 operands, d <= 128 (v_mfma_f32_16x16x32_bf16) ----------------------
// Lane group g takes the features [g L, g L + L), L = ceil(d/32) * 8, eight per
// MFMA step s (steps with 8 s >= L are not issued). The squares of the
// BF16-rounded operands are summed in step and feature order; sum_groups adds
// the four groups' sums.

// Eight features rounded to BF16, their squares added to sq in order.
__device__ __attribute__((always_inline)) inline bf16x8 cvt8_bf16(const float (&v)[8], float& sq) {
    bf16x8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        out[e] = __bf16(v[e]);
        const float r = float(out[e]);
        sq = __builtin_fmaf(r, r, sq);
    }
    return out;
}

// Eight consecutive features k0..k0+7 of one row (zeros past d), rounded to BF16.
template <bool VEC>
__device__ inline bf16x8 load8_bf16(const float* __restrict__ row, bool ok, int64_t k0, int64_t d, float& sq) {
    float v[8];
    if (VEC && ok && k0 + 8 <= d) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(row + k0);
        const f32x4 b = *reinterpret_cast<const f32x4*>(row + k0 + 4);
        v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
        v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (ok && k0 + e < d) ? row[k0 + e] : 0.0f;
    }
    return cvt8_bf16(v, sq);
}

// The column operands of panel p and their inverse norms (zeros past m).
template <bool VEC>
__device__ __attribute__((always_inline)) inline void panel_operands_bf16(const float* __restrict__ Y, int64_t m,
                                                                          int64_t d, int64_t p, bf16x8 (&bv)[4][4],
                                                                          float (&ry)[4]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int64_t L = (d + 31) / 32 * 8;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t col = p * kPanel + b * 16 + (lane & 15);
        const bool ok = col < m;
        const float* yrow = Y + (ok ? col : 0) * d;
        float sb = 0.0f;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            bv[b][s] = bf16x8{};
            if (8 * s < L) bv[b][s] = load8_bf16<VEC>(yrow, ok, g * L + 8 * s, d, sb);
        }
        ry[b] = inv_from_sq(sum_groups(sb));
    }
}

}  // namespace pardtw
