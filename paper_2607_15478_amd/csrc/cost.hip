// a1 + a2 + a7: cosine-distance cost matrix (Sec. IV) as an MFMA GEMM on gfx950.
//
//   C[i,j] = 1 - (<x_i, y_j> * rx_i) * ry_j,   rx_i = 1/|x_i| (0 for a zero frame)
//
// A workgroup of four waves sweeps kTilesPerBlock tiles of 64 rows x 64
// columns down one column panel; each wave owns 16 rows of a tile and issues
// 16x16 MFMA blocks over the feature dimension: v_mfma_f32_16x16x4_f32 for
// FP32 operands, v_mfma_f32_16x16x32_bf16 for BF16 operands (FP32 accumulate
// in both).
//
// Operands: the MFMA sums over all features, so how they are split between
// the four 16-lane groups and the steps is free; each path picks the split its
// loads like (see the tile functions). The squared operands summed over the
// four groups (two cross-lane xors) give every lane the norm of its row and of
// its columns, so the inverse norms come out of the operand registers with no
// extra loads and no workgroup barrier. For d <= 16 (FP32) a workgroup keeps
// its panel's column operands in registers for its whole sweep.
//
// The tile is written either into the DP's panel layout (rows 0-3 then 4-7 of
// each 8-row group, 16 contiguous bytes per column: one 16-byte store per lane
// per 16x16 block) or row-major. For the DP's own use the panel layout can skip
// every 8-row group of a panel outside the band of cells that can lie on a path
// from (0,0) to (N-1,M-1) (the DP never reads those groups): about 70% of the
// matrix for a 5:6 pair. With D = 12 the kernel does 24 flop per
// 4-byte output, far below the MFMA ridge point: it is bound by HBM writes.
#include "batch.h"
#include "cost_slab.h"

namespace pardtw {
namespace {

constexpr int kTileM = 64;
constexpr int kThreads = 256;
constexpr int kTilesPerBlock = 16;  // row tiles swept by one workgroup

// Groups of panel p outside [lo, hi] are not written.
struct GroupSpan {
    int64_t lo, hi;
};

// band: 0 every group, 1 the DTW path band, 2 the subsequence band.
__device__ inline GroupSpan group_span(int band, int64_t p, int64_t n, int64_t m) {
    GroupSpan s;
    s.lo = band == 1 ? band_group_lo(p, n, m) : band == 2 ? sub_group_lo(p, n, m) : 0;
    s.hi = band == 1 ? band_group_hi(p, n, m) : band == 2 ? sub_group_hi(p, n, m) : (int64_t(1) << 62);
    return s;
}

// Whether rows [i0, i0 + rows) touch a written group.
__device__ inline bool rows_written(const GroupSpan& s, int64_t i0, int64_t rows) {
    return i0 / kBpRows <= s.hi && (i0 + rows - 1) / kBpRows >= s.lo;
}

// Store of a wave's 16 rows of a 64-row x 64-column tile: v[b] holds the costs
// of rows 4*(lane/16) + r of column b*16 + lane%16 (the layout of cost_slab.h).
template <bool PANEL>
__device__ __attribute__((always_inline)) inline void store_tile(const f32x4 (&v)[4], int64_t n, int64_t m,
                                                                 float* __restrict__ C, int64_t p, int64_t i0,
                                                                 const GroupSpan& span) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tr0 = 4 * (lane >> 4);  // first of the lane's 4 rows within the wave's 16
    const int64_t ib = i0 + wave * 16 + tr0;
    if constexpr (PANEL) {
        const int64_t G = bp_groups(n);
        const int64_t grp = ib / kBpRows;
        if (grp < G && grp >= span.lo && grp <= span.hi) {
            const int64_t half = (p * G + ib / kBpRows) * 2 + (ib % kBpRows) / 4;
            float* dst = C + half * (kPanel * 4);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int cc = b * 16 + (lane & 15);
                __builtin_nontemporal_store(v[b], reinterpret_cast<f32x4*>(dst + cc * 4));
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = ib + r;
            if (i >= n) continue;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t j = p * kPanel + b * 16 + (lane & 15);
                if (j < m) __builtin_nontemporal_store(v[b][r], C + i * m + j);
            }
        }
    }
}

// FP32, d <= 16: feature k = 4t + g (g = lane/16) at MFMA step t. The panel's
// column operands and their inverse norms stay in registers for the whole
// sweep of the workgroup; each tile loads only its rows.
template <bool PANEL>
__device__ __attribute__((always_inline)) inline void sweep_f32_small(const float* __restrict__ X,
                                                                      const float* __restrict__ Y, int64_t n,
                                                                      int64_t m, int64_t d, float* __restrict__ C,
                                                                      int64_t p, int64_t t0, int tiles,
                                                                      const GroupSpan& span) {
    const int wave = threadIdx.x >> 6;
    float bv[4][4], ry[4];
    panel_operands_f32_small(Y, m, d, p, bv, ry);
    for (int u = 0; u < tiles; ++u) {
        const int64_t i0 = (t0 + u) * kTileM;
        if (i0 >= n) break;
        if (!rows_written(span, i0, kTileM)) continue;
        f32x4 v[4];
        slab_costs_f32_small(X, n, d, i0 + wave * 16, bv, ry, v);
        store_tile<PANEL>(v, n, m, C, p, i0, span);
    }
}

// Any d. FP32: with VEC, lane group g takes the contiguous features
// [g*L, g*L + L), L = ceil(d/16)*4, four per 16-byte load; otherwise feature
// k = 4t + g at step t (neighbouring lanes read neighbouring features). BF16:
// group g takes [g*L, g*L + L), L = ceil(d/32)*8, eight per step.
template <bool BF16, bool PANEL, bool VEC>
__device__ __attribute__((always_inline)) inline void cost_tile(const float* __restrict__ X,
                                                                const float* __restrict__ Y, int64_t n, int64_t m,
                                                                int64_t d, float* __restrict__ C, int64_t p,
                                                                int64_t i0, const GroupSpan& span) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int64_t arow = i0 + wave * 16 + (lane & 15);
    const bool arow_ok = arow < n;
    const float* xrow = X + (arow_ok ? arow : 0) * d;
    const float* yrow[4];
    bool bok[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t col = p * kPanel + b * 16 + (lane & 15);
        bok[b] = col < m;
        yrow[b] = Y + (bok[b] ? col : 0) * d;
    }

    f32x4 acc[4];
    float sa = 0.0f, sb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        sb[b] = 0.0f;
    }
    if constexpr (!BF16 && VEC) {
        const int64_t L = (d + 15) / 16 * 4;
        for (int64_t t = 0; t < L; t += 4) {
            const int64_t k0 = g * L + t;
            f32x4 a = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (arow_ok && k0 < d) a = *reinterpret_cast<const f32x4*>(xrow + k0);  // d % 4 == 0: whole vector
            f32x4 bb[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                bb[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                if (bok[b] && k0 < d) bb[b] = *reinterpret_cast<const f32x4*>(yrow[b] + k0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sa = __builtin_fmaf(a[e], a[e], sa);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    sb[b] = __builtin_fmaf(bb[b][e], bb[b][e], sb[b]);
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], bb[b][e], acc[b], 0, 0, 0);
                }
            }
        }
    } else if constexpr (!BF16) {
        const int64_t T = (d + 3) / 4;
        for (int64_t t = 0; t < T; ++t) {
            const int64_t k = 4 * t + g;
            const float av = (arow_ok && k < d) ? xrow[k] : 0.0f;
            sa = __builtin_fmaf(av, av, sa);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float bv = (bok[b] && k < d) ? yrow[b][k] : 0.0f;
                sb[b] = __builtin_fmaf(bv, bv, sb[b]);
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[b], 0, 0, 0);
            }
        }
    } else {
        const int64_t L = (d + 31) / 32 * 8;
        for (int64_t t = 0; t < L; t += 8) {
            const int64_t k0 = g * L + t;
            const bf16x8 av = load8_bf16<VEC>(xrow, arow_ok, k0, d, sa);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const bf16x8 bv = load8_bf16<VEC>(yrow[b], bok[b], k0, d, sb[b]);
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[b], 0, 0, 0);
            }
        }
    }
    float ry[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) ry[b] = inv_from_sq(sum_groups(sb[b]));
    f32x4 v[4];
    costs_from_acc(acc, inv_from_sq(sum_groups(sa)), ry, v);
    store_tile<PANEL>(v, n, m, C, p, i0, span);
}

// BF16, d <= 128: the panel's column operands (at most four steps of eight
// features per lane group) and their inverse norms are loaded once and kept in
// registers for the whole sweep, instead of once per 64-row tile; the row
// operands, the MFMA steps and their order are cost_tile's, so the costs are
// the same bits.
template <bool PANEL, bool VEC>
__device__ __attribute__((always_inline)) inline void sweep_bf16_small(const float* __restrict__ X,
                                                                       const float* __restrict__ Y, int64_t n,
                                                                       int64_t m, int64_t d, float* __restrict__ C,
                                                                       int64_t p, int64_t t0, int tiles,
                                                                       const GroupSpan& span) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int64_t L = (d + 31) / 32 * 8;  // features per lane group, <= 32
    bf16x8 bv[4][4];
    float ry[4];
    panel_operands_bf16<VEC>(Y, m, d, p, bv, ry);
    for (int u = 0; u < tiles; ++u) {
        const int64_t i0 = (t0 + u) * kTileM;
        if (i0 >= n) break;
        if (!rows_written(span, i0, kTileM)) continue;
        const int64_t arow = i0 + wave * 16 + (lane & 15);
        const bool arow_ok = arow < n;
        const float* xrow = X + (arow_ok ? arow : 0) * d;
        f32x4 acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        float sa = 0.0f;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (8 * s < L) {
                const bf16x8 av = load8_bf16<VEC>(xrow, arow_ok, g * L + 8 * s, d, sa);
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[b][s], acc[b], 0, 0, 0);
            }
        }
        f32x4 v[4];
        costs_from_acc(acc, inv_from_sq(sum_groups(sa)), ry, v);
        store_tile<PANEL>(v, n, m, C, p, i0, span);
    }
}

// FP32 with d % 16 == 0 and 16 < d <= 128: the panel's 64 columns (d floats
// each, rows padded to d + 4 so that 16 lanes reading 16 columns hit distinct
// banks) are staged in LDS once for the workgroup's tiles, and their inverse
// norms computed once, instead of reloading them per 64-row tile. The loads,
// the MFMA steps and their order are cost_tile's, so the costs are the same
// bits.
constexpr int kLdsMaxD = 128;
template <bool PANEL>
__device__ __attribute__((always_inline)) inline void sweep_f32_lds(const float* __restrict__ X,
                                                                    const float* __restrict__ Y, int64_t n,
                                                                    int64_t m, int64_t d, float* __restrict__ C,
                                                                    int64_t p, int64_t t0, int tiles,
                                                                    const GroupSpan& span) {
    __shared__ __attribute__((aligned(16))) float ys[kPanel][kLdsMaxD + 4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    for (int64_t e = threadIdx.x; e < int64_t(kPanel) * d; e += kThreads) {
        const int64_t c = e / d, k = e % d;
        const int64_t col = p * kPanel + c;
        ys[c][k] = col < m ? Y[col * d + k] : 0.0f;
    }
    __syncthreads();
    const int64_t L = (d + 15) / 16 * 4;  // features per lane group (d % 16 == 0: L = d / 4)
    float ry[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float* yc = &ys[b * 16 + (lane & 15)][0];
        float sb = 0.0f;
        for (int64_t t = 0; t < L; t += 4) {
            const f32x4 bb = *reinterpret_cast<const f32x4*>(yc + g * L + t);
#pragma unroll
            for (int e = 0; e < 4; ++e) sb = __builtin_fmaf(bb[e], bb[e], sb);
        }
        ry[b] = inv_from_sq(sum_groups(sb));
    }
    for (int u = 0; u < tiles; ++u) {
        const int64_t i0 = (t0 + u) * kTileM;
        if (i0 >= n) break;
        if (!rows_written(span, i0, kTileM)) continue;
        const int64_t arow = i0 + wave * 16 + (lane & 15);
        const bool arow_ok = arow < n;
        const float* xrow = X + (arow_ok ? arow : 0) * d;
        f32x4 acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        float sa = 0.0f;
        for (int64_t t = 0; t < L; t += 4) {
            const int64_t k0 = g * L + t;
            f32x4 a = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (arow_ok && k0 < d) a = *reinterpret_cast<const f32x4*>(xrow + k0);
            f32x4 bb[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) bb[b] = *reinterpret_cast<const f32x4*>(&ys[b * 16 + (lane & 15)][k0]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sa = __builtin_fmaf(a[e], a[e], sa);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], bb[b][e], acc[b], 0, 0, 0);
            }
        }
        f32x4 v[4];
        costs_from_acc(acc, inv_from_sq(sum_groups(sa)), ry, v);
        store_tile<PANEL>(v, n, m, C, p, i0, span);
    }
}

// A workgroup's sweep: tiles t0 .. t0 + kTilesPerBlock - 1 of panel p. With a
// `band` (panel layout only) the groups outside it are skipped.
template <bool BF16, bool PANEL, bool VEC>
__device__ __attribute__((always_inline)) inline void sweep(const float* __restrict__ X,
                                                            const float* __restrict__ Y, int64_t n, int64_t m,
                                                            int64_t d, float* __restrict__ C, int64_t p, int64_t t0,
                                                            int band) {
    const GroupSpan span = group_span(PANEL ? band : 0, p, n, m);
    if (!rows_written(span, t0 * kTileM, int64_t(kTilesPerBlock) * kTileM)) return;
    if (!BF16 && d <= 16) {
        sweep_f32_small<PANEL>(X, Y, n, m, d, C, p, t0, kTilesPerBlock, span);
        return;
    }
    if constexpr (BF16) {
        if (d <= 128) {
            sweep_bf16_small<PANEL, VEC>(X, Y, n, m, d, C, p, t0, kTilesPerBlock, span);
            return;
        }
    } else if constexpr (VEC) {
        if (d <= kLdsMaxD) {
            sweep_f32_lds<PANEL>(X, Y, n, m, d, C, p, t0, kTilesPerBlock, span);
            return;
        }
    }
    for (int u = 0; u < kTilesPerBlock; ++u) {
        const int64_t i0 = (t0 + u) * kTileM;
        if (i0 >= n) break;
        if (!rows_written(span, i0, kTileM)) continue;
        cost_tile<BF16, PANEL, VEC>(X, Y, n, m, d, C, p, i0, span);
    }
}

// Rows swept by one workgroup.
constexpr int64_t kBlockRows = int64_t(kTileM) * kTilesPerBlock;

// With a band, block (p, y) takes the y-th block of rows from the one holding
// the panel's first band group, so the grid's height is the widest band in
// blocks rather than all of n (21 of 49 blocks of rows for a 50000 x 60000 pair).
template <bool BF16, bool PANEL, bool VEC>
__global__ __launch_bounds__(kThreads) void cost_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                        int64_t n, int64_t m, int64_t d, float* __restrict__ C,
                                                        int band) {
    const int64_t p = blockIdx.x;
    int64_t rb = blockIdx.y;
    if (band != 0) rb += group_span(band, p, n, m).lo * kBpRows / kBlockRows;
    sweep<BF16, PANEL, VEC>(X, Y, n, m, d, C, p, rb * kTilesPerBlock, band);
}

// The grid height for a band: the most blocks of rows that one panel's band
// groups span (at least 1).
int64_t band_grid_rows(int band, int64_t n, int64_t m) {
    int64_t rows = 1;
    const int64_t last = (n - 1) / kBpRows;
    for (int64_t p = 0; p < num_panels(m); ++p) {
        const int64_t lo = band == 1 ? band_group_lo(p, n, m) : sub_group_lo(p, n, m);
        int64_t hi = band == 1 ? band_group_hi(p, n, m) : sub_group_hi(p, n, m);
        if (hi > last) hi = last;
        if (lo > hi) continue;
        const int64_t span = hi * kBpRows / kBlockRows - lo * kBpRows / kBlockRows + 1;
        if (span > rows) rows = span;
    }
    return rows;
}

// Batched form: block t is block t of the batch's numbering; tile_pair[t]
// names its pair, whose blocks are numbered panel-major from pairs[b].tile0.
template <bool BF16, bool VEC>
__global__ __launch_bounds__(kThreads) void cost_batch_kernel(const BatchPair* __restrict__ pairs,
                                                              const int32_t* __restrict__ tile_pair,
                                                              const float* __restrict__ X,
                                                              const float* __restrict__ Y, int64_t d,
                                                              float* __restrict__ Cbase) {
    const int64_t t = blockIdx.x;
    const BatchPair q = pairs[tile_pair[t]];
    const int64_t local = t - q.tile0;
    const int64_t rows_blk = ceil_div(ceil_div(q.n, kTileM), kTilesPerBlock);
    const int64_t p = local / rows_blk;
    const int64_t t0 = (local % rows_blk) * kTilesPerBlock;
    sweep<BF16, true, VEC>(X + q.x_off * d, Y + q.y_off * d, q.n, q.m, d, Cbase + q.c_off, p, t0, q.band);
}

bool vec_ok(const float* X, const float* Y, int64_t d) {
    return d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0;
}

}  // namespace

int64_t cost_blocks(int64_t n, int64_t m) {
    return num_panels(m) * ceil_div(ceil_div(n, kTileM), kTilesPerBlock);
}

pardtw_status cost_batch_launch(const BatchPair* pairs, const int32_t* tile_pair, int64_t tiles, const float* X,
                                const float* Y, int64_t d, pardtw_prec prec, float* Cbase, hipStream_t stream) {
    if (tiles <= 0) return PARDTW_OK;
    if (tiles > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    // packed pairs start at row offsets that keep 16-byte alignment when d % 4 == 0
    const bool vec = vec_ok(X, Y, d);
    const unsigned grid = unsigned(tiles);
    if (prec == PARDTW_PREC_F32 && vec && d % 16 == 0) {
        cost_batch_kernel<false, true><<<grid, kThreads, 0, stream>>>(pairs, tile_pair, X, Y, d, Cbase);
    } else if (prec == PARDTW_PREC_F32) {
        cost_batch_kernel<false, false><<<grid, kThreads, 0, stream>>>(pairs, tile_pair, X, Y, d, Cbase);
    } else if (vec) {
        cost_batch_kernel<true, true><<<grid, kThreads, 0, stream>>>(pairs, tile_pair, X, Y, d, Cbase);
    } else {
        cost_batch_kernel<true, false><<<grid, kThreads, 0, stream>>>(pairs, tile_pair, X, Y, d, Cbase);
    }
    return launch_status();
}

pardtw_status cost_launch(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, pardtw_prec prec,
                          pardtw_layout layout, float* C, hipStream_t stream) {
    const int band = layout == PARDTW_LAYOUT_PANEL_BAND ? 1 : layout == PARDTW_LAYOUT_PANEL_SUBSEQ_BAND ? 2 : 0;
    const int64_t rows_blk = band != 0 ? band_grid_rows(band, n, m) : ceil_div(ceil_div(n, kTileM), kTilesPerBlock);
    if (rows_blk > 65535 || num_panels(m) > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    dim3 grid(unsigned(num_panels(m)), unsigned(rows_blk));
    const bool panel = layout != PARDTW_LAYOUT_ROW;
    const bool vec = vec_ok(X, Y, d);
    if (prec == PARDTW_PREC_F32 && vec && d % 16 == 0) {
        if (panel) cost_kernel<false, true, true><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
        else cost_kernel<false, false, true><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
    } else if (prec == PARDTW_PREC_F32) {
        if (panel) cost_kernel<false, true, false><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
        else cost_kernel<false, false, false><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
    } else if (vec) {
        if (panel) cost_kernel<true, true, true><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
        else cost_kernel<true, false, true><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
    } else {
        if (panel) cost_kernel<true, true, false><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
        else cost_kernel<true, false, false><<<grid, kThreads, 0, stream>>>(X, Y, n, m, d, C, band);
    }
    return launch_status();
}

}  // namespace pardtw

extern "C" size_t pardtw_cost_elems(int64_t n, int64_t m, pardtw_layout layout) {
    if (!pardtw::valid_sizes(n, m)) return 0;
    if (layout == PARDTW_LAYOUT_ROW) return size_t(n) * size_t(m);
    if (layout == PARDTW_LAYOUT_PANEL || layout == PARDTW_LAYOUT_PANEL_BAND ||
        layout == PARDTW_LAYOUT_PANEL_SUBSEQ_BAND)
        return size_t(pardtw::num_panels(m)) * size_t(pardtw::bp_groups(n)) * pardtw::kPanel * pardtw::kBpRows;
    return 0;
}

extern "C" pardtw_status pardtw_band_groups(int64_t n, int64_t m, int64_t p, int64_t* lo, int64_t* hi) {
    if (!lo || !hi || !pardtw::valid_sizes(n, m) || p < 0 || p >= pardtw::num_panels(m)) return PARDTW_ERR_INVALID_ARG;
    const int64_t G = pardtw::bp_groups(n);
    const int64_t l = pardtw::band_group_lo(p, n, m), h = pardtw::band_group_hi(p, n, m);
    *lo = l < G ? l : G;
    *hi = h < G - 1 ? h : G - 1;
    return PARDTW_OK;
}

extern "C" pardtw_status pardtw_subseq_band_groups(int64_t n, int64_t m, int64_t p, int64_t* lo, int64_t* hi) {
    if (!lo || !hi || !pardtw::valid_sizes(n, m) || p < 0 || p >= pardtw::num_panels(m)) return PARDTW_ERR_INVALID_ARG;
    const int64_t G = pardtw::bp_groups(n);
    const int64_t l = pardtw::sub_group_lo(p, n, m), h = pardtw::sub_group_hi(p, n, m);
    *lo = l < G ? l : G;
    *hi = h < G - 1 ? h : G - 1;
    return PARDTW_OK;
}

extern "C" pardtw_status pardtw_cost(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                     pardtw_prec prec, pardtw_layout layout, float* C, hipStream_t stream) {
    if (!X || !Y || !C || !pardtw::valid_sizes(n, m) || d <= 0 || d > (int64_t(1) << 20))
        return PARDTW_ERR_INVALID_ARG;
    if (prec != PARDTW_PREC_F32 && prec != PARDTW_PREC_BF16) return PARDTW_ERR_UNSUPPORTED;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL && layout != PARDTW_LAYOUT_PANEL_BAND &&
        layout != PARDTW_LAYOUT_PANEL_SUBSEQ_BAND)
        return PARDTW_ERR_UNSUPPORTED;
    return pardtw::cost_launch(X, Y, n, m, d, prec, layout, C, stream);
}
