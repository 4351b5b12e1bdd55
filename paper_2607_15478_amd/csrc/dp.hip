// a3: the ParDTW accumulated-cost dynamic program on gfx950.
//
// Recurrence (Sec. V step set {(1,1),(1,2),(2,1)}, weights {2,3,3}):
//   D[i,j] = min(D[i-1,j-1] + 2C, D[i-1,j-2] + 3C, D[i-2,j-1] + 3C),  D[0,0] = C[0,0].
// A cell needs only the two rows above it (equivalently: anti-diagonal k needs
// diagonals k-2 and k-3, which is why the paper keeps four diagonal buffers,
// Sec. II-D). So a whole row of a column panel is one step of independent
// cells.
//
// Schedule. Columns are cut into 64-wide panels; one wavefront owns a panel,
// one lane per column, and walks its rows top to bottom keeping D of the last
// row and the shifted D of the row before in registers. Row i of lane l needs
// D[i-1][j-1], D[i-1][j-2] and D[i-2][j-1]: two wave_shr:1 DPP moves per row,
// whose lane 0 is fed the two boundary columns of the panel to the left.
// Panel p trails panel p-1 by a few rows, so the sweep front is a staircase
// along the anti-diagonal of the (row, panel) grid and every panel is active
// at once.
//
// A workgroup holds NW compute waves (NW consecutive panels) and one helper
// wave. Boundary columns pass between the compute waves of a workgroup through
// LDS rings, 8 rows at a time; between workgroups they pass through global
// records {float D, uint32 epoch} written with agent-scope 64-bit atomic stores
// and polled, several chunks per round trip, by the helper wave of the next
// workgroup, so no side issues a cache-flushing fence. Workgroups take groups
// of panels from an atomic ticket in increasing order; a group only waits on
// lower tickets, held by running workgroups, so the sweep always makes
// progress whatever the number of resident workgroups.
//
// Memory traffic per cell: 4 bytes of cost read and 1 byte of backtrace code
// written. In the panel layout a lane reads its column's 8 costs of a chunk
// as two 16-byte loads and writes its 8 codes as one 8-byte store; a wave's
// chunk is 2 KB of contiguous cost and 512 contiguous bytes of codes.
#include "common.h"

namespace pardtw {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = kBpRows;  // rows per synchronisation chunk (= packed group)
constexpr int kRing = 16;        // LDS ring depth, in chunks
constexpr int kPfPanel = 8;      // cost prefetch distance in chunks, panel layout
constexpr int kPfRow = 4;        // the same for the row-major layout (8 loads per chunk)
constexpr int kHelperWin = 4;    // chunks polled per helper round trip (64 lanes)
constexpr int kMaxNW = 4;

struct DpShared {
    int super;
    int prog[kMaxNW + 1];  // ring w: chunks published by its producer
    int cons[kMaxNW + 1];  // ring w: chunks released by its consumer
    // ring[w][slot][c][r] = D[8k + r][64p - 2 + c] for chunk k, slot = k % kRing
    float ring[kMaxNW + 1][kRing][2][kChunk];
};

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

struct DpArgs {
    const float* C;
    uint8_t* bp;
    float* total;
    int32_t* status;
    DpWsHeader* hdr;
    uint64_t* rec;  // [P][G*8][2] boundary records
    int64_t n, m;
    int64_t G;      // 8-row groups per panel
    int P;          // number of panels
    int S;          // number of panel groups (= ceil(P / NW))
};

enum { kOutNone = 0, kOutLocal = 1, kOutGlobal = 2 };

template <bool PANEL>
__device__ __attribute__((always_inline)) inline void load_chunk(const DpArgs& a, int p, int lane, int64_t k, float (&cb)[kChunk]) {
    if constexpr (PANEL) {
        const f32x4* src = reinterpret_cast<const f32x4*>(a.C + ((int64_t(p) * a.G + k) * kLanes + lane) * kChunk);
        const f32x4 v0 = __builtin_nontemporal_load(src);
        const f32x4 v1 = __builtin_nontemporal_load(src + 1);
        cb[0] = v0[0]; cb[1] = v0[1]; cb[2] = v0[2]; cb[3] = v0[3];
        cb[4] = v1[0]; cb[5] = v1[1]; cb[6] = v1[2]; cb[7] = v1[3];
    } else {
        const int64_t j = int64_t(p) * kPanel + lane;
        const bool colv = j < a.m;
#pragma unroll
        for (int r = 0; r < kChunk; ++r) {
            const int64_t i = k * kChunk + r;
            cb[r] = (colv && i < a.n) ? __builtin_nontemporal_load(a.C + i * a.m + j) : 0.0f;
        }
    }
}

template <int NW, bool PANEL, bool HAVE_LEFT, int OUT>
__device__ __attribute__((always_inline)) inline void compute_wave(const DpArgs& a, DpShared& sh, int wave, int p, uint32_t epoch) {
    const int lane = threadIdx.x & 63;
    const int64_t G = a.G;  // chunks per panel (rows padded to a multiple of 8)
    const float kInf = __builtin_inff();
    const int bcol = lane - (kLanes - 2);  // 0 / 1 on the two boundary lanes
    float* rin = &sh.ring[wave][0][0][0];
    float* rout = &sh.ring[wave + 1][0][0][0];
    uint64_t* rec_out = a.rec + (size_t(p) * size_t(G) * kChunk) * 2;
    uint64_t* bp_out = reinterpret_cast<uint64_t*>(a.bp) + int64_t(p) * G * kLanes + lane;

    constexpr int kPf = PANEL ? kPfPanel : kPfRow;
    float cbuf[kPf][kChunk];
#pragma unroll
    for (int u = 0; u < kPf; ++u)
        if (u < G) load_chunk<PANEL>(a, p, lane, u, cbuf[u]);

    // D[i-1][j] and D[i-2][j-1]. The origin is produced by the general rule
    // through a virtual D[-2][-1] = -2 C[0][0]: fma(3, C00, -2 C00) = C00
    // exactly, and that value is used by no other cell.
    float d1 = kInf;
    float s1p = (p == 0 && lane == 0) ? -2.0f * cbuf[0][0] : kInf;
    // left boundary D[i-1][64p-2], D[i-1][64p-1] for the first row of the chunk
    float e0 = kInf, e1 = kInf;
    int prog_seen = 0, cons_seen = 0;
    const int64_t last = G - 1;
    const int rlast = int((a.n - 1) % kChunk);
    float dlast = kInf;

    for (int64_t k0 = 0; k0 < G; k0 += kPf) {
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            const int64_t k = k0 + u;
            if (k >= G) break;
            const int slot = int(k % kRing);

            float lv0[kChunk], lv1[kChunk];
            if constexpr (HAVE_LEFT) {
                if (prog_seen <= k) {
                    int v;
                    while ((v = lds_get(&sh.prog[wave])) <= k) __builtin_amdgcn_s_sleep(1);
                    prog_seen = v;
                }
                compiler_order();
                const f32x4* src = reinterpret_cast<const f32x4*>(rin + slot * 2 * kChunk);
                const f32x4 a0 = src[0], a1 = src[1], b0 = src[2], b1 = src[3];
                lv0[0] = a0[0]; lv0[1] = a0[1]; lv0[2] = a0[2]; lv0[3] = a0[3];
                lv0[4] = a1[0]; lv0[5] = a1[1]; lv0[6] = a1[2]; lv0[7] = a1[3];
                lv1[0] = b0[0]; lv1[1] = b0[1]; lv1[2] = b0[2]; lv1[3] = b0[3];
                lv1[4] = b1[0]; lv1[5] = b1[1]; lv1[6] = b1[2]; lv1[7] = b1[3];
                compiler_order();
                if (lane == 0) lds_put(&sh.cons[wave], int(k + 1));
            } else {
#pragma unroll
                for (int r = 0; r < kChunk; ++r) { lv0[r] = kInf; lv1[r] = kInf; }
            }

            uint32_t lo = 0, hi = 0;
            float best_r[kChunk];
#pragma unroll
            for (int r = 0; r < kChunk; ++r) {
                const float c = cbuf[u][r];
                const float s1 = shift_in(d1, r == 0 ? e1 : lv1[r - 1]);  // D[i-1][j-1]
                const float s2 = shift_in(s1, r == 0 ? e0 : lv0[r - 1]);  // D[i-1][j-2]
                const float c0 = __builtin_fmaf(2.0f, c, s1);
                const float c1 = __builtin_fmaf(3.0f, c, s2);
                const float c2 = __builtin_fmaf(3.0f, c, s1p);
                const float best = __builtin_fminf(__builtin_fminf(c0, c1), c2);
                uint32_t code = (c1 == best) ? 1u : 2u;
                code = (c0 == best) ? 0u : code;
                code = (best == kInf) ? 3u : code;
                if (r < 4) lo |= code << (8 * r); else hi |= code << (8 * (r - 4));
                d1 = best;
                s1p = s1;
                best_r[r] = best;
            }
            e0 = lv0[kChunk - 1];
            e1 = lv1[kChunk - 1];
            if (p == 0 && k == 0) lo = (lane == 0) ? ((lo & ~0xffu) | 3u) : lo;  // the origin's code
            __builtin_nontemporal_store(uint64_t(lo) | (uint64_t(hi) << 32), bp_out + k * kLanes);

            if constexpr (OUT == kOutLocal) {
                if (cons_seen < k + 1 - kRing) {
                    int v;
                    while ((v = lds_get(&sh.cons[wave + 1])) < k + 1 - kRing) __builtin_amdgcn_s_sleep(1);
                    cons_seen = v;
                }
                compiler_order();
                if (bcol >= 0) {
                    f32x4* dst = reinterpret_cast<f32x4*>(rout + (slot * 2 + bcol) * kChunk);
                    dst[0] = f32x4{best_r[0], best_r[1], best_r[2], best_r[3]};
                    dst[1] = f32x4{best_r[4], best_r[5], best_r[6], best_r[7]};
                }
                compiler_order();
                if (lane == 0) lds_put(&sh.prog[wave + 1], int(k + 1));
            } else if constexpr (OUT == kOutGlobal) {
                if (bcol >= 0) {
#pragma unroll
                    for (int r = 0; r < kChunk; ++r) {
                        const uint64_t v = (uint64_t(epoch) << 32) | uint64_t(__float_as_uint(best_r[r]));
                        __hip_atomic_store(rec_out + (k * kChunk + r) * 2 + bcol, v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            if (k == last) {
#pragma unroll
                for (int r = 0; r < kChunk; ++r) dlast = (r == rlast) ? best_r[r] : dlast;
            }

            if (k + kPf < G) load_chunk<PANEL>(a, p, lane, k + kPf, cbuf[u]);
        }
    }
    if (int64_t(p) * kPanel + lane == a.m - 1) {
        *a.total = dlast;
        *a.status = dlast == kInf ? PARDTW_PAIR_INFEASIBLE : PARDTW_PAIR_OK;
    }
}

// Helper wave: copies the boundary columns of panel pl (the last panel of the
// previous group, computed by another workgroup) from the global records into
// LDS ring 0. Each poll covers up to kHelperWin chunks (16 records each) and
// publishes every leading chunk whose epoch tags are all present.
__device__ __attribute__((always_inline)) inline void helper_wave(const DpArgs& a, DpShared& sh, int pl, uint32_t epoch) {
    const int lane = threadIdx.x & 63;
    const int64_t G = a.G;
    const uint64_t* rec = a.rec + (size_t(pl) * size_t(G) * kChunk) * 2;
    float* ring = &sh.ring[0][0][0][0];
    const int q = lane >> 4;           // chunk within the poll window
    const int row = (lane & 15) >> 1;  // row within that chunk
    const int col = lane & 1;
    int cons_seen = 0;
    for (int64_t k = 0; k < G;) {
        const int64_t kq = k + q;
        const bool want = kq < G;
        uint64_t v = 0;
        bool ok = true;
        if (want) {
            v = __hip_atomic_load(rec + (kq * kChunk + row) * 2 + col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = uint32_t(v >> 32) == epoch;
        }
        const uint64_t good = __builtin_amdgcn_ballot_w64(ok);
        int ready = 0;
        while (ready < kHelperWin && ((good >> (16 * ready)) & 0xffffull) == 0xffffull && k + ready < G) ++ready;
        if (ready == 0) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        if (cons_seen < k + ready - kRing) {
            int c;
            while ((c = lds_get(&sh.cons[0])) < k + ready - kRing) __builtin_amdgcn_s_sleep(1);
            cons_seen = c;
        }
        compiler_order();
        if (q < ready) ring[((int(kq % kRing)) * 2 + col) * kChunk + row] = __uint_as_float(uint32_t(v));
        compiler_order();
        if (lane == 0) lds_put(&sh.prog[0], int(k + ready));
        k += ready;
    }
}

template <int NW, bool PANEL>
__device__ __attribute__((always_inline)) inline void run_compute(const DpArgs& a, DpShared& sh, int wave, int p, uint32_t epoch) {
    const bool left = p > 0;
    const int out = (p + 1 >= a.P) ? kOutNone : (wave < NW - 1 ? kOutLocal : kOutGlobal);
    if (left) {
        if (out == kOutLocal) compute_wave<NW, PANEL, true, kOutLocal>(a, sh, wave, p, epoch);
        else if (out == kOutGlobal) compute_wave<NW, PANEL, true, kOutGlobal>(a, sh, wave, p, epoch);
        else compute_wave<NW, PANEL, true, kOutNone>(a, sh, wave, p, epoch);
    } else {
        if (out == kOutLocal) compute_wave<NW, PANEL, false, kOutLocal>(a, sh, wave, p, epoch);
        else if (out == kOutGlobal) compute_wave<NW, PANEL, false, kOutGlobal>(a, sh, wave, p, epoch);
        else compute_wave<NW, PANEL, false, kOutNone>(a, sh, wave, p, epoch);
    }
}

template <int NW, bool PANEL>
__global__ __launch_bounds__(kLanes*(NW + 1)) void dp_kernel(DpArgs a) {
    __shared__ DpShared sh;
    const int wave = threadIdx.x / kLanes;
    const uint32_t epoch = __hip_atomic_load(&a.hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) {
            sh.super = int(atomicAdd(&a.hdr->ticket, 1u));
            for (int w = 0; w <= NW; ++w) { sh.prog[w] = 0; sh.cons[w] = 0; }
        }
        __syncthreads();
        const int q = sh.super;
        if (q >= a.S) break;
        const int p0 = q * NW;
        if (wave < NW) {
            const int p = p0 + wave;
            if (p < a.P) run_compute<NW, PANEL>(a, sh, wave, p, epoch);
        } else if (p0 > 0) {
            helper_wave(a, sh, p0 - 1, epoch);
        }
        __syncthreads();
    }
}

__global__ void dp_prepare(DpWsHeader* hdr) {
    hdr->epoch = hdr->epoch + 1;
    hdr->ticket = 0;
}

int choose_nw(int P) {
    // One compute wave per SIMD: prefer 4 panels per workgroup while that still
    // gives most CUs a workgroup, fall back to fewer for narrow problems.
    if (P >= 4 * 200) return 4;
    if (P >= 2 * 200) return 2;
    return 1;
}

template <int NW>
void launch_nw(const DpArgs& a, bool panel, int grid, hipStream_t stream) {
    if (panel) dp_kernel<NW, true><<<grid, kLanes * (NW + 1), 0, stream>>>(a);
    else dp_kernel<NW, false><<<grid, kLanes * (NW + 1), 0, stream>>>(a);
}

}  // namespace

size_t dp_workspace_bytes_impl(int64_t n, int64_t m) {
    return sizeof(DpWsHeader) + size_t(num_panels(m)) * size_t(bp_groups(n)) * kChunk * 2 * sizeof(uint64_t);
}

pardtw_status dp_launch(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                        float* total, int32_t* status, void* ws, int nw_override, hipStream_t stream) {
    DpArgs a;
    a.C = C;
    a.bp = bp;
    a.total = total;
    a.status = status;
    a.hdr = reinterpret_cast<DpWsHeader*>(ws);
    a.rec = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(ws) + sizeof(DpWsHeader));
    a.n = n;
    a.m = m;
    a.G = bp_groups(n);
    a.P = int(num_panels(m));
    const int nw = nw_override > 0 ? nw_override : choose_nw(a.P);
    a.S = int(ceil_div(a.P, nw));
    int dev = 0, cus = 0;
    PARDTW_HIP_TRY(hipGetDevice(&dev));
    PARDTW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = a.S < cus ? a.S : cus;
    const bool panel = layout == PARDTW_LAYOUT_PANEL;
    dp_prepare<<<1, 1, 0, stream>>>(a.hdr);
    switch (nw) {
        case 1: launch_nw<1>(a, panel, grid, stream); break;
        case 2: launch_nw<2>(a, panel, grid, stream); break;
        case 4: launch_nw<4>(a, panel, grid, stream); break;
        default: return PARDTW_ERR_UNSUPPORTED;
    }
    return launch_status();
}

}  // namespace pardtw

extern "C" size_t pardtw_dp_workspace_bytes(int64_t n, int64_t m) {
    if (!pardtw::valid_sizes(n, m)) return 0;
    return pardtw::dp_workspace_bytes_impl(n, m);
}

extern "C" size_t pardtw_bp_bytes(int64_t n, int64_t m) {
    if (!pardtw::valid_sizes(n, m)) return 0;
    return size_t(pardtw::num_panels(m)) * size_t(pardtw::bp_groups(n)) * pardtw::kLanes * pardtw::kBpRows;
}

extern "C" pardtw_status pardtw_dp(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                                   float* total, int32_t* pair_status, void* workspace,
                                   size_t workspace_bytes, hipStream_t stream) {
    if (!C || !bp || !total || !pair_status || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL) return PARDTW_ERR_UNSUPPORTED;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(C, layout, n, m, bp, total, pair_status, workspace, 0, stream);
}

extern "C" pardtw_status pardtw_dp_ex(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                                      float* total, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                                      int32_t panels_per_workgroup, hipStream_t stream) {
    if (!C || !bp || !total || !pair_status || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL) return PARDTW_ERR_UNSUPPORTED;
    if (panels_per_workgroup != 0 && panels_per_workgroup != 1 && panels_per_workgroup != 2 &&
        panels_per_workgroup != 4)
        return PARDTW_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(C, layout, n, m, bp, total, pair_status, workspace, panels_per_workgroup, stream);
}
