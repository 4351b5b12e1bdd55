// Compensated total of a path (the accumulation in two-float arithmetic
// proposed against FP32 rounding of long sums).
//
// The DP accumulates D[i,j] = D[pred] + w C[i,j] in FP32, rounding once per
// step, so along a path of L cells its total drifts by up to about L FP32
// rounding errors of the growing partial sums. Its decisions fix the path;
// the path's cost (Sec. V: the start cell's cost plus, per step, the step's
// weight times the cost of the cell it lands on) is then re-summed here with
// every term added exactly into a (hi, lo) pair of floats: a product w c is
// split exactly into p + e with an FMA, and each addition's rounding error is
// recovered with Knuth's two-sum and carried in lo. The costs are the cosine
// distances of the FP32 features (a zero frame costs 1), evaluated as half the
// squared distance of the normalised frames so that their FP32 error stays
// relative to the distance. The result equals the path's exact cost up to
// those FP32 costs and one final rounding.
#include "common.h"

namespace pardtw {
namespace {

struct F2 {
    float hi, lo;
};

// s + e == a + b exactly (Knuth).
__device__ inline F2 two_sum(float a, float b) {
    const float s = a + b;
    const float bv = s - a;
    const float av = s - bv;
    return {s, (a - av) + (b - bv)};
}

// x + v, with the rounding error of the addition kept in lo.
__device__ inline F2 f2_add(F2 x, float v) {
    const F2 s = two_sum(x.hi, v);
    return two_sum(s.hi, s.lo + x.lo);
}

__device__ inline F2 f2_add(F2 x, F2 y) {
    const F2 s = two_sum(x.hi, y.hi);
    return two_sum(s.hi, s.lo + (x.lo + y.lo));
}

// The cosine distance of one cell, as half the squared distance of the unit
// vectors: 1 - <u, v> = |u - v|^2 / 2 for |u| = |v| = 1. Computed this way the
// rounding error is relative to the (small) distance, whereas 1 - <u, v> loses
// an ulp of 1 to cancellation when u and v are nearly parallel. N features are
// read through x(k), y(k) (zeros past d add nothing).
template <int N, class VX, class VY>
__device__ inline float cell_cost(const VX& x, const VY& y, int64_t d) {
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int64_t k = 0; k < (N > 0 ? N : d); ++k) {
        sx = __builtin_fmaf(x(k), x(k), sx);
        sy = __builtin_fmaf(y(k), y(k), sy);
    }
    if (!(sx > 0.0f) || !(sy > 0.0f)) return 1.0f;  // a zero frame: the normalised vector is 0
    const float rx = 1.0f / __builtin_sqrtf(sx), ry = 1.0f / __builtin_sqrtf(sy);
    float s = 0.0f;
#pragma unroll
    for (int64_t k = 0; k < (N > 0 ? N : d); ++k) {
        const float t = __builtin_fmaf(x(k), rx, -(y(k) * ry));
        s = __builtin_fmaf(t, t, s);
    }
    return 0.5f * s;
}

constexpr int kTotalThreads = 256;  // four waves, one per SIMD, with room for kCells rows in registers
constexpr int kTotalBlocks = 256;   // one per CU: the path is cut into this many contiguous pieces
constexpr int kCells = 8;   // path cells per thread and round, their loads issued together
constexpr int kRegD = 16;   // features held in registers (d <= 16, d % 4 == 0); other rows are read in place

// Weight of the step into path cell l (1 at the start).
__device__ inline float step_weight(const int2* __restrict__ pp, int64_t l, int2 cur) {
    if (l == 0) return 1.0f;
    const int2 prev = pp[l - 1];
    return (cur.x - prev.x == 1 && cur.y - prev.y == 1) ? 2.0f : 3.0f;
}

// Adds the (hi, lo) pairs of a block's threads in a tree through LDS; thread 0
// gets the sum.
__device__ inline F2 block_sum(F2* part, F2 acc) {
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kTotalThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) part[threadIdx.x] = f2_add(part[threadIdx.x], part[threadIdx.x + s]);
        __syncthreads();
    }
    return part[0];
}

// Block b sums piece b of the path (cells [b q, (b + 1) q), q = ceil(len /
// kTotalBlocks)): each thread a strided share, kCells at a time, then the
// block's pairs in a tree. The pieces depend only on the length, so the
// result does not depend on the schedule.
__global__ __launch_bounds__(kTotalThreads) void path_total_kernel(const float* __restrict__ X,
                                                                   const float* __restrict__ Y, int64_t d,
                                                                   const int32_t* __restrict__ path,
                                                                   const int32_t* __restrict__ path_len,
                                                                   F2* partial) {
    __shared__ F2 part[kTotalThreads];
    const int64_t len = *path_len;
    const int64_t q = (len + kTotalBlocks - 1) / kTotalBlocks;
    const int64_t beg = int64_t(blockIdx.x) * q;
    const int64_t end = beg + q < len ? beg + q : len;
    const int2* pp = reinterpret_cast<const int2*>(path);
    F2 acc = {0.0f, 0.0f};
    for (int64_t l0 = beg + threadIdx.x; l0 < end; l0 += int64_t(kTotalThreads) * kCells) {
        int2 cell[kCells];
        float w[kCells], c[kCells];
#pragma unroll
        for (int u = 0; u < kCells; ++u) {
            const int64_t l = l0 + int64_t(u) * kTotalThreads;
            cell[u] = l < end ? pp[l] : int2{0, 0};
            w[u] = l < end ? step_weight(pp, l, cell[u]) : 0.0f;
        }
        if (d <= kRegD && d % 4 == 0) {
            // rows of whole 16-byte vectors (X and Y start 16-byte aligned)
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 xv[kCells][kRegD / 4], yv[kCells][kRegD / 4];
#pragma unroll
            for (int u = 0; u < kCells; ++u)
#pragma unroll
                for (int q = 0; q < kRegD / 4; ++q) {
                    const bool in = 4 * q < d;
                    xv[u][q] = in ? reinterpret_cast<const f4*>(X + int64_t(cell[u].x) * d)[q] : f4{0, 0, 0, 0};
                    yv[u][q] = in ? reinterpret_cast<const f4*>(Y + int64_t(cell[u].y) * d)[q] : f4{0, 0, 0, 0};
                }
#pragma unroll
            for (int u = 0; u < kCells; ++u)
                c[u] = cell_cost<kRegD>([&](int64_t k) { return xv[u][k >> 2][k & 3]; },
                                        [&](int64_t k) { return yv[u][k >> 2][k & 3]; }, d);
        } else {
#pragma unroll
            for (int u = 0; u < kCells; ++u) {
                const float* x = X + int64_t(cell[u].x) * d;
                const float* y = Y + int64_t(cell[u].y) * d;
                c[u] = cell_cost<0>([&](int64_t k) { return x[k]; }, [&](int64_t k) { return y[k]; }, d);
            }
        }
#pragma unroll
        for (int u = 0; u < kCells; ++u) {
            const float p = w[u] * c[u];
            const float e = __builtin_fmaf(w[u], c[u], -p);  // w c = p + e exactly
            acc = f2_add(acc, p);
            acc.lo += e;
        }
    }
    const F2 sum = block_sum(part, acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// The kTotalBlocks pieces, added in a tree; +inf for an empty path.
__global__ __launch_bounds__(kTotalThreads) void path_total_final_kernel(const F2* __restrict__ partial,
                                                                         const int32_t* __restrict__ path_len,
                                                                         float* total) {
    static_assert(kTotalBlocks == kTotalThreads, "one piece per thread");
    __shared__ F2 part[kTotalThreads];
    const F2 sum = block_sum(part, partial[threadIdx.x]);
    if (threadIdx.x == 0) *total = *path_len > 0 ? sum.hi + sum.lo : __builtin_inff();
}

}  // namespace
}  // namespace pardtw

extern "C" size_t pardtw_path_total_bytes(void) { return pardtw::kTotalBlocks * sizeof(pardtw::F2); }

extern "C" pardtw_status pardtw_path_total(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                           const int32_t* path, const int32_t* path_len, float* total,
                                           void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!X || !Y || !path || !path_len || !total || !workspace || !pardtw::valid_sizes(n, m) || d <= 0)
        return PARDTW_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 8 != 0) return PARDTW_ERR_INVALID_ARG;
    if (workspace_bytes < pardtw_path_total_bytes()) return PARDTW_ERR_WORKSPACE;
    pardtw::F2* partial = reinterpret_cast<pardtw::F2*>(workspace);
    pardtw::path_total_kernel<<<pardtw::kTotalBlocks, pardtw::kTotalThreads, 0, stream>>>(X, Y, d, path, path_len,
                                                                                          partial);
    pardtw::path_total_final_kernel<<<1, pardtw::kTotalThreads, 0, stream>>>(partial, path_len, total);
    return pardtw::launch_status();
}
