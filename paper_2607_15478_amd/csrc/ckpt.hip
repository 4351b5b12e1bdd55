// Checkpointed backtrace: the exact DTW path without the n x m code matrix,
// for lengths whose codes would not fit in memory. Sec. II-D cites the
// divide-and-conquer answer to the same limit (linear memory, cost recomputed);
// this is its two-level form, sized for one GPU's HBM.
//
// Forward: the fused DP (costs computed in the sweep) stores no codes, only D
// of the two rows before every block of K rows (pardtw_dp_fused_ckpt, in
// dp.hip): 8 m / K bytes per row instead of m.
//
// Backward (here): one workgroup walks the blocks from the last. Above a path
// cell (ie, je) in block [r0, r0 + K), the path reaches row r at a column in
// the cone je - 2(ie - r) <= c <= je - ceil((ie - r) / 2): every step moves
// one or two columns per row, and at least half a column per row. The cone
// holds every predecessor of its cells down to row r0, and the two
// checkpoint rows above r0 hold the rest, so recomputing D over it from those
// rows gives every cell on the path the D, and so the code, of the full
// sweep. The recomputation runs the sweep's own instructions: the row step of
// dp_step.h, one wave per 64-column panel with the same boundary handoff, and
// the same MFMA slab and row norms for the costs (cost_slab.h). Its 2-bit
// codes stay in LDS, and wave 0 follows them 32 rows at a time with the
// lane-parallel window trace (trace.h) until the path leaves the block; the
// cell it leaves to starts the next block.
//
// Work: the cones cover about 3/4 K^2 cells per block, about n K in all,
// against n m for the sweep; memory: the checkpoints, 8 n m / K bytes.
#include "dp_step.h"
#include "split.h"
#include "trace.h"

namespace pardtw {
namespace {

constexpr int kCkGroups = kCkMaxRows / kChunk;         // 8-row groups of a block
constexpr int kCkPanels = 2 * kCkMaxRows / kPanel + 2;  // panels a window can span
constexpr int kCkCols = kCkPanels * kPanel;
constexpr int kCkThreads = kCkPanels * kLanes;          // one wave per window panel

struct CkShared {
    alignas(16) float xs[kCkMaxRows][16];  // the block's feature rows, zero past n and d
    alignas(16) float rx[kCkMaxRows];      // their inverse norms, zero past n
    // per wave: the costs of one 16-row slab, two chunks in the sweep's ring layout
    alignas(16) float tr[kCkPanels][2][kChunk * kLanes];
    // ring[w][k][c][r] = D[r0 + 8k + r][64(plo + w) + 62 + c]
    float ring[kCkPanels][kCkGroups][2][kChunk];
    // codes[k][cc]: 2 bits per row (row r0 + 8k + r at bits 2r) of column 64 plo + cc
    uint16_t codes[kCkGroups][kCkCols];
    int prog[kCkPanels];  // chunks wave w has published
    int ie, je, len, fail;
};

struct CkArgs {
    const float* X;
    const float* Y;
    int64_t n, m, d;
    int K;
    const float* ckpt;
    int64_t stride;  // floats per checkpoint row
    const int32_t* status;
    int32_t* path;
    int32_t* path_len;
};

// Four 1-byte codes (one word, code r in byte r) to 2 bits each, code r at bits 2r.
__device__ inline uint32_t compact4(uint32_t x) {
    x = (x | (x >> 6)) & 0x000F000Fu;
    return (x | (x >> 12)) & 0xFFu;
}

// A window wave's inputs, loaded at the start of a block together with the
// feature rows: the panel's column operands and the D values it starts from,
// D[r0-1][j] and D[r0-2][j-1], and the left boundary D[r0-1][64p-2],
// D[r0-1][64p-1].
struct WaveStart {
    float bv[4][4], ry[4];
    float d1, s1p, e0, e1;
};

__device__ __attribute__((always_inline)) inline void load_start(const CkArgs& a, int wave, int r0, int p,
                                                                 WaveStart& w) {
    const int lane = threadIdx.x & 63;
    const float kInf = __builtin_inff();
    panel_operands_f32_small(a.Y, a.m, a.d, p, w.bv, w.ry);
    w.d1 = kInf;
    w.s1p = kInf;
    w.e0 = kInf;
    w.e1 = kInf;
    // The first wave's left boundary is never needed: its columns lie left of
    // every predecessor of a window cell.
    if (r0 > 0) {
        const int64_t col = int64_t(p) * kPanel + lane;
        const float* c2 = a.ckpt + int64_t(2 * (r0 / a.K - 1)) * a.stride;  // row r0 - 2
        const float* c1 = c2 + a.stride;                                     // row r0 - 1
        w.d1 = c1[col];
        w.s1p = col >= 1 ? c2[col - 1] : kInf;
        if (wave > 0) {
            w.e0 = c1[col - lane - 2];
            w.e1 = c1[col - lane - 1];
        }
    }
}

// The window of block [r0, ie] ending at column je, on wave `wave` (panel plo + wave).
__device__ void window_wave(CkShared& sh, const WaveStart& st, int wave, int r0, int ie, int je, int plo,
                            int nch) {
    const int lane = threadIdx.x & 63;
    const int p = plo + wave;
    const float kInf = __builtin_inff();
    float d1 = st.d1, s1p = st.s1p, e0 = st.e0, e1 = st.e1;
    // The panel holds window cells on rows rmin .. rmax only: the cone's left
    // edge je - 2(ie - r) passes the panel's last column at rmax, its right
    // edge je - ceil((ie - r) / 2) its first column at rmin.
    const int over = je - (p * kPanel + kPanel - 1);
    const int rmax = over > 0 ? ie - (over + 1) / 2 : ie;
    const int kend = rmax >= r0 ? (rmax - r0) / kChunk : -1;
    const int rmin = ie - 2 * (je - p * kPanel);
    const int kbeg = rmin > r0 ? (rmin - r0) / kChunk : 0;
    const bool origin = r0 == 0 && p == 0 && lane == 0;
    const int kq = lane >> 5, half = (lane >> 4) & 1, tcol = lane & 15;
    int left_seen = 0;
    if (kbeg > 0 && kbeg <= kend) {
        // Rows above chunk kbeg hold no window cell of this panel, so the window
        // cells of its first rows take their predecessors from the panel to the
        // left (wave > 0 here: the first panel starts at row r0): rows R-1 and
        // R-2 of its last two columns, R = r0 + 8 kbeg.
        while (left_seen < kbeg) {
            left_seen = lds_get(&sh.prog[wave - 1]);
            if (left_seen < kbeg) __builtin_amdgcn_s_sleep(1);
        }
        compiler_order();
        e0 = sh.ring[wave - 1][kbeg - 1][0][kChunk - 1];
        e1 = sh.ring[wave - 1][kbeg - 1][1][kChunk - 1];
        const float sl = sh.ring[wave - 1][kbeg - 1][1][kChunk - 2];
        d1 = kInf;
        s1p = lane == 0 ? sl : kInf;
    }
    for (int k = kbeg; k <= kend; ++k) {
        if ((k & 1) == 0 || k == kbeg) {
            // rows r0 + 8(k & ~1) .. + 15: the sweep's slab (r0 is a multiple of 16)
            const int rs = kChunk * (k & ~1);
            float av[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) av[t] = sh.xs[rs + (lane & 15)][4 * t + (lane >> 4)];
            const f32x4 rx4 = *reinterpret_cast<const f32x4*>(&sh.rx[rs + 4 * (lane >> 4)]);
            f32x4 acc[4], v[4];
            slab_acc_f32_small(16, av, st.bv, acc);  // every step: the same sums (zeros past d)
            costs_from_acc_rx(acc, rx4, st.ry, v);
            float* dst = &sh.tr[wave][kq][half * (kLanes * 4)];
#pragma unroll
            for (int b = 0; b < 4; ++b) *reinterpret_cast<f32x4*>(dst + (b * 16 + tcol) * 4) = v[b];
            compiler_order();
        }
        float cb[kChunk];
        {
            const f32x4* src = reinterpret_cast<const f32x4*>(&sh.tr[wave][k & 1][0]) + lane;
            const f32x4 v0 = src[0], v1 = src[kLanes];
            cb[0] = v0[0]; cb[1] = v0[1]; cb[2] = v0[2]; cb[3] = v0[3];
            cb[4] = v1[0]; cb[5] = v1[1]; cb[6] = v1[2]; cb[7] = v1[3];
        }
        if (k == 0 && origin) s1p = -2.0f * cb[0];  // D[0][0] = C[0][0], as in the sweep
        float lv0[kChunk], lv1[kChunk];
        if (wave > 0) {
            while (left_seen <= k) {
                left_seen = lds_get(&sh.prog[wave - 1]);
                if (left_seen <= k) __builtin_amdgcn_s_sleep(1);
            }
            compiler_order();
#pragma unroll
            for (int r = 0; r < kChunk; ++r) {
                lv0[r] = sh.ring[wave - 1][k][0][r];
                lv1[r] = sh.ring[wave - 1][k][1][r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < kChunk; ++r) lv0[r] = lv1[r] = kInf;
        }
        uint32_t lo, hi;
        float best_r[kChunk];
        dp_rows<false>(cb, lv0, lv1, e0, e1, d1, s1p, lo, hi, best_r);
        if (k == 0 && origin) lo = (lo & ~0xffu) | 3u;
        e0 = lv0[kChunk - 1];
        e1 = lv1[kChunk - 1];
        sh.codes[k][wave * kPanel + lane] = uint16_t(compact4(lo) | (compact4(hi) << 8));
        if (lane >= kLanes - 2) {
#pragma unroll
            for (int r = 0; r < kChunk; ++r) sh.ring[wave][k][lane - (kLanes - 2)][r] = best_r[r];
        }
        compiler_order();
        lds_put(&sh.prog[wave], k + 1);
    }
    // rows past kend hold no window cell of this panel: its right neighbour
    // may read whatever its ring holds there
    compiler_order();
    lds_put(&sh.prog[wave], nch);
}

// Wave 0: follows the codes from (i, j) until the path leaves rows r0 .. ie
// or reaches the origin, 32 rows at a time: lane b holds column j - b of rows
// i-31 .. i, and the window trace resolves them at once. Rows above r0 (the
// block before) are not traced: the cell the path enters there starts the
// next block. The k-th cell of the walk goes to out[k] (`forward`) or to
// out[cap - 1 - k].
__device__ void walk_block(CkShared& sh, int r0, int plo, int cap, int32_t* out, bool forward) {
    const int lane = threadIdx.x & 63;
    int i = __builtin_amdgcn_readfirstlane(sh.ie);
    int j = __builtin_amdgcn_readfirstlane(sh.je);
    int len = __builtin_amdgcn_readfirstlane(sh.len);
    bool done = false, fail = false;
    const int cbase = plo * kPanel;
    while (i >= r0 && !done && !fail) {
        const int rr = i - r0;
        // rows rr-31 .. rr: groups g0 .. g0+4, row x at bit 2(x - 8 g0) of lo
        // and 2(x - 8 g0) - 16 of hi; groups below 0 are the block before
        const int g0 = (rr - 31) >> 3;  // floor
        const int cc = j - lane - cbase;
        uint32_t w[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            const int g = g0 + t;
            w[t] = (cc >= 0 && g >= 0 && g <= (rr >> 3)) ? uint32_t(sh.codes[g][cc]) : 0u;
        }
        const int s2 = 2 * (rr - 8 * g0);  // in [62, 76]
        const uint64_t lo = uint64_t(w[0]) | (uint64_t(w[1]) << 16) | (uint64_t(w[2]) << 32) | (uint64_t(w[3]) << 48);
        const uint64_t hi = uint64_t(w[1]) | (uint64_t(w[2]) << 16) | (uint64_t(w[3]) << 32) | (uint64_t(w[4]) << 48);
        const WindowMasks wm = window_masks(uint32_t(hi >> (s2 - 46)), uint32_t(lo >> (s2 - 62)));
        const uint32_t live = rr >= 31 ? ~0u : ~0u << (31 - rr);  // rows a <= rr
        const uint32_t on = trace_window_live(wm, live, lane);
        const uint64_t has = __builtin_amdgcn_ballot_w64(on != 0);  // lane 0 holds the start cell
        const int last = 63 - __builtin_clzll(has);                   // the last cell marked
        const int la = __builtin_clz(uint32_t(__builtin_amdgcn_readlane(int(on), last)));
        const uint32_t lrows = uint32_t(__builtin_amdgcn_readlane(int(wm.two_rows), last));
        const uint32_t lcols = uint32_t(__builtin_amdgcn_readlane(int(wm.two_cols), last));
        int cnt = __builtin_popcountll(has);
        int da, db;
        if (la > rr) {
            // entered the block before: that cell is not written here
            --cnt;
            da = la;
            db = last;
        } else if (((lrows & lcols) >> (31 - la)) & 1u) {
            // code 3: the origin ends the path
            done = true;
            fail = i - la != 0 || j - last != 0;
            da = la;
            db = last;
        } else {
            // left through the 32nd row
            da = la + 1 + int((lrows >> (31 - la)) & 1u);
            db = last + 1 + int((lcols >> (31 - la)) & 1u);
            if (da < 32) fail = true;
        }
        if (len + cnt > cap) fail = true;
        if (fail) break;
        if (on != 0 && (lane != last || cnt == __builtin_popcountll(has))) {
            const int idx = int(__builtin_amdgcn_mbcnt_hi(uint32_t(has >> 32),
                                                          __builtin_amdgcn_mbcnt_lo(uint32_t(has), 0u)));
            const int64_t pos = forward ? int64_t(len + idx) : int64_t(cap) - 1 - (len + idx);
            out[2 * pos] = i - __builtin_clz(on);
            out[2 * pos + 1] = j - lane;
        }
        len += cnt;
        i -= da;
        j -= db;
    }
    if (!done && !fail && i < 0) fail = true;
    if (lane == 0) {
        sh.ie = (done || fail) ? -1 : i;
        sh.je = j;
        sh.len = len;
        sh.fail = fail ? 1 : 0;
    }
}

// Fills the boundary rings with +inf once per kernel (the blocks' windows
// then keep them consistent).
__device__ void ck_init(CkShared& sh) {
    for (int e = threadIdx.x; e < kCkPanels * kCkGroups * 2 * kChunk; e += kCkThreads)
        (&sh.ring[0][0][0][0])[e] = __builtin_inff();
}

// Walks the path from (i0, j0) block by block (each block's window recomputed
// from its checkpoints, then traced) until it reaches the origin or, with
// stop_row >= 0, a cell on a row <= stop_row, which goes to *ex (a segment of
// the split walk; stop_row + 1 is a block's first row). Cells go to out as
// walk_block writes them. Returns the number of cells, 0 if the walk failed
// (or, with stop_row >= 0, reached the origin). Called by the whole workgroup.
__device__ int ck_walk(const CkArgs& a, CkShared& sh, int i0, int j0, int stop_row, int32_t* out, bool forward,
                       int cap, int2* ex) {
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) {
        sh.ie = i0;
        sh.je = j0;
        sh.len = 0;
        sh.fail = 0;
    }
    __syncthreads();
    constexpr int kXPer = kCkMaxRows * 16 / kCkThreads + 1;  // feature loads per thread
    for (;;) {
        const int ie = __builtin_amdgcn_readfirstlane(sh.ie);
        const int je = __builtin_amdgcn_readfirstlane(sh.je);
        if (ie < 0 || ie <= stop_row) break;
        const int r0 = ie - ie % a.K;
        const int A = ie - r0;
        const int nch = A / kChunk + 1;  // chunks holding rows r0 .. ie
        const int cl = je - 2 * A - 2;   // leftmost column a window cell reads
        const int plo = cl > 0 ? cl / kPanel : 0;
        const int phi = je / kPanel;
        const int xrows = 16 * ((nch + 1) / 2);  // whole slabs
        const bool active = plo + wave <= phi;
        // one round trip: the wave's operands and start values, and the feature rows
        WaveStart st;
        if (active) load_start(a, wave, r0, plo + wave, st);
        float xv[kXPer];
#pragma unroll
        for (int t = 0; t < kXPer; ++t) {
            const int e = tid + t * kCkThreads;
            const int64_t row = r0 + (e >> 4);
            const int k = e & 15;
            xv[t] = (e < xrows * 16 && row < a.n && k < a.d) ? a.X[row * a.d + k] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < kXPer; ++t) {
            const int e = tid + t * kCkThreads;
            if (e < xrows * 16) sh.xs[e >> 4][e & 15] = xv[t];
        }
        if (tid < kCkPanels) sh.prog[tid] = 0;
        __syncthreads();
        // the row norms as the sweep computes them (zero past n, where the rows are zero)
        for (int rr = tid; rr < xrows; rr += kCkThreads) {
            float x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = sh.xs[rr][k];
            sh.rx[rr] = inv_norm16(x);
        }
        __syncthreads();
        if (active) window_wave(sh, st, wave, r0, ie, je, plo, nch);
        __syncthreads();
        if (wave == 0) walk_block(sh, r0, plo, cap, out, forward);
        __syncthreads();
    }
    const int ie = __builtin_amdgcn_readfirstlane(sh.ie);
    const int je = __builtin_amdgcn_readfirstlane(sh.je);
    const bool fail = sh.fail != 0 || (stop_row >= 0 && ie < 0);
    if (ex) *ex = make_int2(ie, je);
    return fail ? 0 : sh.len;
}

__global__ __launch_bounds__(kCkThreads) void ckpt_backtrace_kernel(CkArgs a) {
    __shared__ CkShared sh;
    const int tid = threadIdx.x;
    const int cap = int(a.n < a.m ? a.n : a.m);
    if (*a.status != PARDTW_PAIR_OK) {
        if (tid == 0) *a.path_len = 0;
        return;
    }
    ck_init(sh);
    const int len = ck_walk(a, sh, int(a.n - 1), int(a.m - 1), -1, a.path, false, cap, nullptr);
    // the path was written backwards from entry cap-1: move it to the front
    const int64_t base = int64_t(cap) - len;
    int2* pp = reinterpret_cast<int2*>(a.path);
    constexpr int kPer = 8;
    for (int64_t q0 = 0; q0 < len; q0 += int64_t(kCkThreads) * kPer) {
        int2 v[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int64_t q = q0 + t * kCkThreads + tid;
            if (q < len) v[t] = pp[base + q];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int64_t q = q0 + t * kCkThreads + tid;
            if (q < len) pp[q] = v[t];
        }
        __syncthreads();
    }
    if (tid == 0) *a.path_len = len;
}

// ---- Split walk over the blocks (split.h) ------------------------------------
// Segments are runs of whole blocks (R a multiple of K), each walked by one
// workgroup with ck_walk from its start down to its first row.
__device__ SegInfo ck_segment(const CkArgs& a, CkShared& sh, SegInfo& res, const SplitArgs& sp, int s, int si,
                              int sj, SegInfo* out) {
    int2 ex;
    const int len = ck_walk(a, sh, si, sj, seg_stop_row(s, sp.R), sp.cells + int64_t(s) * sp.R * 2, true, sp.R, &ex);
    if (threadIdx.x == 0) {
        const SegInfo r = seg_info(si, sj, ex.x, ex.y, len);
        *out = r;
        res = r;
    }
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kCkThreads) void ck_seg_round_kernel(CkArgs a, SplitArgs sp, int round) {
    __shared__ CkShared sh;
    __shared__ SegInfo res;
    if (*a.status != PARDTW_PAIR_OK) return;
    ck_init(sh);
    split_round(sp, blockIdx.x, round, [&](int s, int si, int sj, SegInfo* out) {
        return ck_segment(a, sh, res, sp, s, si, sj, out);
    });
}

__global__ __launch_bounds__(kCkThreads) void ck_seg_finish_kernel(CkArgs a, SplitArgs sp, int fin) {
    __shared__ CkShared sh;
    __shared__ SegInfo res;
    __shared__ SegInfo sinfo[kSegMaxCount];
    if (*a.status != PARDTW_PAIR_OK) {
        if (threadIdx.x == 0) *a.path_len = 0;
        return;
    }
    ck_init(sh);
    split_finish(sp, sinfo, fin, int(a.n < a.m ? a.n : a.m), a.path_len, [&](int s, int si, int sj, SegInfo* out) {
        return ck_segment(a, sh, res, sp, s, si, sj, out);
    });
}

__global__ __launch_bounds__(256) void ck_seg_copy_kernel(SplitArgs sp, int fin, const int32_t* __restrict__ path_len,
                                                          int32_t* __restrict__ path) {
    if (*path_len <= 0) return;
    split_copy(sp, blockIdx.x, fin, path);
}

constexpr int kCkSegRounds = 3;

// Segments of at least four blocks, at most kSegMaxCount of them.
void ck_seg_shape(int64_t n, int K, int& R, int& S) {
    const int64_t blocks = ceil_div(ceil_div(n, int64_t(kSegMaxCount)), int64_t(K));
    R = int(K * (blocks > 4 ? blocks : 4));
    S = int(ceil_div(n, int64_t(R)));
}

size_t ck_seg_bytes(int64_t n, int K) {
    int R, S;
    ck_seg_shape(n, K, R, S);
    return size_t(2) * S * sizeof(SegInfo) + size_t(S) * R * 2 * sizeof(int32_t);
}

}  // namespace
}  // namespace pardtw

extern "C" size_t pardtw_ckpt_bytes(int64_t n, int64_t m, int32_t rows_per_block) {
    if (!pardtw::valid_sizes(n, m) || rows_per_block < 16 || rows_per_block > pardtw::kCkMaxRows ||
        rows_per_block % 16)
        return 0;
    return size_t(pardtw::ckpt_floats(n, m, rows_per_block)) * sizeof(float);
}

extern "C" size_t pardtw_ckpt_backtrace_parallel_bytes(int64_t n, int64_t m, int32_t rows_per_block) {
    if (!pardtw::valid_sizes(n, m) || rows_per_block < 16 || rows_per_block > pardtw::kCkMaxRows ||
        rows_per_block % 16)
        return 0;
    return pardtw::ck_seg_bytes(n, rows_per_block);
}

extern "C" pardtw_status pardtw_ckpt_backtrace(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                               int32_t rows_per_block, const float* ckpt, size_t ckpt_bytes,
                                               const int32_t* pair_status, int32_t* path, int32_t* path_len,
                                               hipStream_t stream) {
    if (!X || !Y || !pair_status || !path || !path_len || !pardtw::valid_sizes(n, m) || d <= 0)
        return PARDTW_ERR_INVALID_ARG;
    if (d > 16) return PARDTW_ERR_UNSUPPORTED;
    if (rows_per_block < 16 || rows_per_block > pardtw::kCkMaxRows || rows_per_block % 16)
        return PARDTW_ERR_INVALID_ARG;
    const int64_t floats = pardtw::ckpt_floats(n, m, rows_per_block);
    if (floats > 0 && (!ckpt || ckpt_bytes < size_t(floats) * sizeof(float))) return PARDTW_ERR_WORKSPACE;
    pardtw::CkArgs a;
    a.X = X;
    a.Y = Y;
    a.n = n;
    a.m = m;
    a.d = d;
    a.K = rows_per_block;
    a.ckpt = ckpt;
    a.stride = pardtw::num_panels(m) * pardtw::kPanel;
    a.status = pair_status;
    a.path = path;
    a.path_len = path_len;
    pardtw::ckpt_backtrace_kernel<<<1, pardtw::kCkThreads, 0, stream>>>(a);
    return pardtw::launch_status();
}

extern "C" pardtw_status pardtw_ckpt_backtrace_parallel(const float* X, const float* Y, int64_t n, int64_t m,
                                                        int64_t d, int32_t rows_per_block, const float* ckpt,
                                                        size_t ckpt_bytes, const int32_t* pair_status, int32_t* path,
                                                        int32_t* path_len, void* workspace, size_t workspace_bytes,
                                                        hipStream_t stream) {
    if (!X || !Y || !pair_status || !path || !path_len || !pardtw::valid_sizes(n, m) || d <= 0)
        return PARDTW_ERR_INVALID_ARG;
    if (d > 16) return PARDTW_ERR_UNSUPPORTED;
    if (rows_per_block < 16 || rows_per_block > pardtw::kCkMaxRows || rows_per_block % 16)
        return PARDTW_ERR_INVALID_ARG;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 16 != 0 || reinterpret_cast<uintptr_t>(path) % 8 != 0)
        return PARDTW_ERR_INVALID_ARG;
    const int64_t floats = pardtw::ckpt_floats(n, m, rows_per_block);
    if (floats > 0 && (!ckpt || ckpt_bytes < size_t(floats) * sizeof(float))) return PARDTW_ERR_WORKSPACE;
    if (workspace_bytes < pardtw::ck_seg_bytes(n, rows_per_block)) return PARDTW_ERR_WORKSPACE;
    pardtw::CkArgs a;
    a.X = X;
    a.Y = Y;
    a.n = n;
    a.m = m;
    a.d = d;
    a.K = rows_per_block;
    a.ckpt = ckpt;
    a.stride = pardtw::num_panels(m) * pardtw::kPanel;
    a.status = pair_status;
    a.path = path;
    a.path_len = path_len;
    pardtw::SplitArgs sp;
    sp.n = int(n);
    sp.m = int(m);
    sp.end = int(m - 1);
    sp.sub = 0;
    pardtw::ck_seg_shape(n, rows_per_block, sp.R, sp.S);
    if (sp.S <= 2) {
        pardtw::ckpt_backtrace_kernel<<<1, pardtw::kCkThreads, 0, stream>>>(a);
        return pardtw::launch_status();
    }
    sp.info = reinterpret_cast<pardtw::SegInfo*>(workspace);
    sp.cells = reinterpret_cast<int32_t*>(sp.info + 2 * sp.S);
    for (int r = 0; r < pardtw::kCkSegRounds; ++r)
        pardtw::ck_seg_round_kernel<<<sp.S, pardtw::kCkThreads, 0, stream>>>(a, sp, r);
    const int fin = (pardtw::kCkSegRounds - 1) & 1;
    pardtw::ck_seg_finish_kernel<<<1, pardtw::kCkThreads, 0, stream>>>(a, sp, fin);
    pardtw::ck_seg_copy_kernel<<<sp.S, 256, 0, stream>>>(sp, fin, path_len, path);
    return pardtw::launch_status();
}
