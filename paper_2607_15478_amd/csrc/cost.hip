// a1 + a2 + a7: cosine-distance cost matrix (Sec. IV) as an MFMA GEMM on gfx950.
//
//   C[i,j] = 1 - (<x_i, y_j> * rx_i) * ry_j,   rx_i = 1/|x_i| (0 for a zero frame)
//
// One workgroup computes a 64-row x 64-column tile, i.e. 64 rows of one column
// panel. Each of its four waves owns 16 rows and issues 16x16 MFMA blocks over
// the feature dimension: v_mfma_f32_16x16x4_f32 for FP32 operands,
// v_mfma_f32_16x16x32_bf16 for BF16 operands (FP32 accumulate in both). The
// inverse norms of the tile's 64 rows and 64 columns are computed in the same
// workgroup into LDS. The tile is written either into the DP's panel layout
// (one contiguous 16 KB block) or row-major.
//
// With D = 12 the kernel does 24 flop per 4-byte output, far below the MFMA
// ridge point, so it is bound by HBM writes; the MFMA keeps the arithmetic off
// the VALU so the stores stream at full rate.
#include "batch.h"

namespace pardtw {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTileM = 64;
constexpr int kThreads = 256;

template <bool BF16>
__device__ inline float operand(float v) {
    if constexpr (BF16) return float(__bf16(v));
    return v;
}

template <bool BF16>
__device__ inline float inv_norm(const float* row, int64_t d) {
    float s = 0.0f;
    for (int64_t k = 0; k < d; ++k) {
        const float v = operand<BF16>(row[k]);
        s = __builtin_fmaf(v, v, s);
    }
    return s > 0.0f ? 1.0f / __builtin_sqrtf(s) : 0.0f;
}

// One 64-row x 64-column tile: rows [i0, i0+64) of column panel p.
template <bool BF16, bool PANEL>
__device__ __attribute__((always_inline)) inline void cost_tile(const float* __restrict__ X,
                                                                const float* __restrict__ Y, int64_t n, int64_t m,
                                                                int64_t d, float* __restrict__ C, int64_t p,
                                                                int64_t i0, float (&rx)[kTileM], float (&ry)[kPanel]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t j0 = p * kPanel;

    if (tid < kTileM) {
        const int64_t i = i0 + tid;
        rx[tid] = i < n ? inv_norm<BF16>(X + i * d, d) : 0.0f;
    } else if (tid < kTileM + kPanel) {
        const int64_t j = j0 + (tid - kTileM);
        ry[tid - kTileM] = j < m ? inv_norm<BF16>(Y + j * d, d) : 0.0f;
    }

    // MFMA operand coordinates: A row = lane%16, B column = lane%16, K group = lane/16
    const int64_t arow = i0 + wave * 16 + (lane & 15);
    const bool arow_ok = arow < n;
    const int kg = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    if constexpr (!BF16) {
        for (int64_t k0 = 0; k0 < d; k0 += 4) {
            const int64_t k = k0 + kg;
            const float av = (arow_ok && k < d) ? X[arow * d + k] : 0.0f;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t col = j0 + b * 16 + (lane & 15);
                const float bv = (col < m && k < d) ? Y[col * d + k] : 0.0f;
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[b], 0, 0, 0);
            }
        }
    } else {
        for (int64_t k0 = 0; k0 < d; k0 += 32) {
            bf16x8 av;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t k = k0 + kg * 8 + e;
                av[e] = __bf16((arow_ok && k < d) ? X[arow * d + k] : 0.0f);
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t col = j0 + b * 16 + (lane & 15);
                bf16x8 bv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int64_t k = k0 + kg * 8 + e;
                    bv[e] = __bf16((col < m && k < d) ? Y[col * d + k] : 0.0f);
                }
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[b], 0, 0, 0);
            }
        }
    }
    __syncthreads();

    // Output of a 16x16 block: lane holds column lane%16 of rows 4*(lane/16) + r,
    // r = 0..3. In the panel layout those four rows of one column are 16
    // contiguous bytes (a half-group), so each lane writes one 16-byte vector
    // per block and the 16 lanes of a row quad cover 256 contiguous bytes.
    const int tr0 = wave * 16 + 4 * (lane >> 4);  // first of the lane's 4 tile rows
    const int64_t ib = i0 + tr0;
    if constexpr (PANEL) {
        const int64_t G = bp_groups(n);
        if (ib / kBpRows < G) {
            const int64_t half = (p * G + ib / kBpRows) * 2 + (ib % kBpRows) / 4;
            float* dst = C + half * (kPanel * 4);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int cc = b * 16 + (lane & 15);
                const float sy = ry[cc];
                f32x4 v;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = 1.0f - (acc[b][r] * rx[tr0 + r]) * sy;
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst + cc * 4));
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = ib + r;
            if (i >= n) continue;
            const float sx = rx[tr0 + r];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int cc = b * 16 + (lane & 15);
                const int64_t j = j0 + cc;
                if (j < m) __builtin_nontemporal_store(1.0f - (acc[b][r] * sx) * ry[cc], C + i * m + j);
            }
        }
    }
}

template <bool BF16, bool PANEL>
__global__ __launch_bounds__(kThreads) void cost_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                        int64_t n, int64_t m, int64_t d, float* __restrict__ C) {
    __shared__ float rx[kTileM];
    __shared__ float ry[kPanel];
    cost_tile<BF16, PANEL>(X, Y, n, m, d, C, blockIdx.x, int64_t(blockIdx.y) * kTileM, rx, ry);
}

// Batched form: block t is tile t of the batch; tile_pair[t] names its pair,
// whose tiles are numbered panel-major from pairs[b].tile0.
template <bool BF16>
__global__ __launch_bounds__(kThreads) void cost_batch_kernel(const BatchPair* __restrict__ pairs,
                                                              const int32_t* __restrict__ tile_pair,
                                                              const float* __restrict__ X,
                                                              const float* __restrict__ Y, int64_t d,
                                                              float* __restrict__ Cbase) {
    __shared__ float rx[kTileM];
    __shared__ float ry[kPanel];
    const int64_t t = blockIdx.x;
    const BatchPair q = pairs[tile_pair[t]];
    const int64_t local = t - q.tile0;
    const int64_t tiles_m = ceil_div(q.n, kTileM);
    cost_tile<BF16, true>(X + q.x_off * d, Y + q.y_off * d, q.n, q.m, d, Cbase + q.c_off, local / tiles_m,
                          (local % tiles_m) * kTileM, rx, ry);
}

}  // namespace

pardtw_status cost_batch_launch(const BatchPair* pairs, const int32_t* tile_pair, int64_t tiles, const float* X,
                                const float* Y, int64_t d, pardtw_prec prec, float* Cbase, hipStream_t stream) {
    if (tiles <= 0) return PARDTW_OK;
    if (tiles > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    if (prec == PARDTW_PREC_F32)
        cost_batch_kernel<false><<<unsigned(tiles), kThreads, 0, stream>>>(pairs, tile_pair, X, Y, d, Cbase);
    else
        cost_batch_kernel<true><<<unsigned(tiles), kThreads, 0, stream>>>(pairs, tile_pair, X, Y, d, Cbase);
    return launch_status();
}

pardtw_status cost_launch(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, pardtw_prec prec,
                          pardtw_layout layout, float* C, hipStream_t stream) {
    const int64_t tiles_m = ceil_div(n, kTileM);
    if (tiles_m > 65535) return PARDTW_ERR_UNSUPPORTED;
    dim3 grid(unsigned(num_panels(m)), unsigned(tiles_m));
    const bool panel = layout == PARDTW_LAYOUT_PANEL;
    if (prec == PARDTW_PREC_F32) {
        if (panel) cost_kernel<false, true><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C);
        else cost_kernel<false, false><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C);
    } else {
        if (panel) cost_kernel<true, true><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C);
        else cost_kernel<true, false><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C);
    }
    return launch_status();
}

}  // namespace pardtw

extern "C" size_t pardtw_cost_elems(int64_t n, int64_t m, pardtw_layout layout) {
    if (!pardtw::valid_sizes(n, m)) return 0;
    if (layout == PARDTW_LAYOUT_ROW) return size_t(n) * size_t(m);
    if (layout == PARDTW_LAYOUT_PANEL)
        return size_t(pardtw::num_panels(m)) * size_t(pardtw::bp_groups(n)) * pardtw::kPanel * pardtw::kBpRows;
    return 0;
}

extern "C" pardtw_status pardtw_cost(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                     pardtw_prec prec, pardtw_layout layout, float* C, hipStream_t stream) {
    if (!X || !Y || !C || !pardtw::valid_sizes(n, m) || d <= 0 || d > (int64_t(1) << 20))
        return PARDTW_ERR_INVALID_ARG;
    if (prec != PARDTW_PREC_F32 && prec != PARDTW_PREC_BF16) return PARDTW_ERR_UNSUPPORTED;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL) return PARDTW_ERR_UNSUPPORTED;
    return pardtw::cost_launch(X, Y, n, m, d, prec, layout, C, stream);
}
