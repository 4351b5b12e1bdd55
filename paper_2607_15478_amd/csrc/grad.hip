// a6: gradient of the DTW cost along the optimal path (the paper motivates
// backpropagating through the optimal alignment path, Sec. I).
//
// With the path P held fixed, J = sum_{(i,j) in P} w_ij * c(x_i, y_j) where
// w = 1 at (0,0) and otherwise the weight (2, 3, 3) of the step landing on
// (i,j), and c = 1 - <u, v>, u = x/|x|, v = y/|y|:
//   dc/dx = -(v - <u,v> u) / |x|,   dc/dy = -(u - <u,v> v) / |y|.
// Every step advances both coordinates, so a row or column appears at most
// once on a path: each path cell owns its output rows and no atomics are
// needed. One wavefront per path cell, lanes over the feature dimension.
#include "batch.h"

namespace pardtw {
namespace {

__device__ inline float wave_sum(float v) {
    // butterfly over the 64 lanes
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct GradPair {
    const float* X;
    const float* Y;
    const int32_t* path;
    const int32_t* path_len;
    const float* g;
    float* dX;
    float* dY;
    int64_t n, m, cap;
};

__global__ __launch_bounds__(256) void zero_kernel(float* __restrict__ a, int64_t count) {
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < count;
         k += int64_t(gridDim.x) * blockDim.x)
        a[k] = 0.0f;
}

__device__ void grad_cell(const GradPair& q, int64_t l, int64_t d, int lane) {
    const int64_t i = q.path[2 * l], j = q.path[2 * l + 1];
    float w = 1.0f;
    if (l > 0) {
        const int64_t di = i - q.path[2 * (l - 1)], dj = j - q.path[2 * (l - 1) + 1];
        w = (di == 1 && dj == 1) ? 2.0f : 3.0f;
    }
    const float* x = q.X + i * d;
    const float* y = q.Y + j * d;
    float sx = 0.0f, sy = 0.0f, sxy = 0.0f;
    for (int64_t k = lane; k < d; k += kLanes) {
        const float a = x[k], b = y[k];
        sx = __builtin_fmaf(a, a, sx);
        sy = __builtin_fmaf(b, b, sy);
        sxy = __builtin_fmaf(a, b, sxy);
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sxy = wave_sum(sxy);
    if (!(sx > 0.0f) || !(sy > 0.0f)) return;  // zero frame: cost is the constant 1
    const float nx = __builtin_sqrtf(sx), ny = __builtin_sqrtf(sy);
    const float rx = 1.0f / nx, ry = 1.0f / ny;
    const float uv = sxy * rx * ry;
    const float gw = *q.g * w;
    for (int64_t k = lane; k < d; k += kLanes) {
        const float u = x[k] * rx, v = y[k] * ry;
        q.dX[i * d + k] = -gw * (v - uv * u) * rx;
        q.dY[j * d + k] = -gw * (u - uv * v) * ry;
    }
}

// grid.x covers path cells (one wave each, 4 waves per block).
__global__ __launch_bounds__(256) void grad_kernel(GradPair q, int64_t d) {
    const int lane = threadIdx.x & 63;
    const int64_t len = *q.path_len;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x / kLanes);
    for (int64_t l = int64_t(blockIdx.x) * (blockDim.x / kLanes) + (threadIdx.x >> 6); l < len; l += waves)
        grad_cell(q, l, d, lane);
}

pardtw_status grad_launch_single(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                 const int32_t* path, const int32_t* path_len, const float* g, float* dX,
                                 float* dY, hipStream_t stream) {
    zero_kernel<<<1024, 256, 0, stream>>>(dX, n * d);
    zero_kernel<<<1024, 256, 0, stream>>>(dY, m * d);
    GradPair q{X, Y, path, path_len, g, dX, dY, n, m, n < m ? n : m};
    const int64_t cap = q.cap;
    const unsigned blocks = unsigned(ceil_div(cap, 4) < 4096 ? ceil_div(cap, 4) : 4096);
    grad_kernel<<<dim3(blocks, 1), 256, 0, stream>>>(q, d);
    return launch_status();
}

// Batched form: grid.y = pair; the plan's descriptors give each pair's rows
// in the packed features and its path, so the launch needs no per-call setup.
__global__ __launch_bounds__(256) void grad_batch_kernel(const BatchPair* __restrict__ pairs, const float* X,
                                                         const float* Y, const int32_t* paths,
                                                         const int32_t* path_len, const float* g, float* dX,
                                                         float* dY, int64_t d) {
    const int b = blockIdx.y;
    const BatchPair pr = pairs[b];
    if (!pr.feasible) return;
    GradPair q{X + pr.x_off * d, Y + pr.y_off * d, paths + 2 * pr.path_off, path_len + b, g + b,
               dX + pr.x_off * d, dY + pr.y_off * d, pr.n, pr.m, pr.n < pr.m ? pr.n : pr.m};
    const int lane = threadIdx.x & 63;
    const int64_t len = *q.path_len;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x / kLanes);
    for (int64_t l = int64_t(blockIdx.x) * (blockDim.x / kLanes) + (threadIdx.x >> 6); l < len; l += waves)
        grad_cell(q, l, d, lane);
}

}  // namespace

pardtw_status grad_batch_launch(const BatchPair* pairs, int32_t batch, int64_t max_cap, int64_t d, const float* X,
                                const float* Y, const int32_t* paths, const int32_t* path_len, const float* g,
                                float* dX, int64_t dX_count, float* dY, int64_t dY_count, hipStream_t stream) {
    zero_kernel<<<2048, 256, 0, stream>>>(dX, dX_count);
    zero_kernel<<<2048, 256, 0, stream>>>(dY, dY_count);
    if (batch <= 0 || max_cap <= 0) return launch_status();
    const unsigned blocks = unsigned(ceil_div(max_cap, 4) < 1024 ? ceil_div(max_cap, 4) : 1024);
    grad_batch_kernel<<<dim3(blocks, unsigned(batch)), 256, 0, stream>>>(pairs, X, Y, paths, path_len, g, dX, dY,
                                                                          d);
    return launch_status();
}

}  // namespace pardtw

extern "C" pardtw_status pardtw_path_grad(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                          const int32_t* path, const int32_t* path_len, const float* g_total,
                                          float* dX, float* dY, hipStream_t stream) {
    if (!X || !Y || !path || !path_len || !g_total || !dX || !dY || !pardtw::valid_sizes(n, m) || d <= 0)
        return PARDTW_ERR_INVALID_ARG;
    return pardtw::grad_launch_single(X, Y, n, m, d, path, path_len, g_total, dX, dY, stream);
}
