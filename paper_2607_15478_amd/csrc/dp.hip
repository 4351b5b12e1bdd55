// a3: the ParDTW accumulated-cost dynamic program on gfx950.
//
// Recurrence (Sec. V step set {(1,1),(1,2),(2,1)}, weights {2,3,3}):
//   D[i,j] = min(D[i-1,j-1] + 2C, D[i-1,j-2] + 3C, D[i-2,j-1] + 3C),  D[0,0] = C[0,0].
// A cell needs only the two rows above it (equivalently: anti-diagonal k needs
// diagonals k-2 and k-3, the paper's four diagonal buffers, Sec. II-D). So a
// whole row of a column panel is one step of independent cells.
//
// Schedule. Columns are cut into 64-wide panels; one wavefront owns a panel,
// one lane per column, and walks its rows top to bottom keeping D of the last
// two rows in registers. Row i of lane l needs D[i-1][j-1], D[i-1][j-2] and
// D[i-2][j-1]: two wave_shr:1 DPP moves per row, with lane 0 fed the two
// boundary columns of the panel to the left. Panel p therefore trails panel
// p-1 by a few rows: the sweep front is a staircase along the anti-diagonal
// of the (row, panel) grid, with every panel active at once.
//
// A workgroup holds NW compute waves (NW consecutive panels) plus one helper
// wave. Boundary columns between the compute waves of a workgroup go through
// an LDS ring; between workgroups they go through global records
// {float D, uint32 epoch} written with agent-scope 64-bit atomic stores and
// polled by the helper wave of the next workgroup, so neither side issues a
// cache-flushing fence. Workgroups take groups of panels from an atomic ticket
// in increasing order; a group only waits on lower tickets, which are held by
// running workgroups, so the sweep always makes progress whatever the number
// of resident workgroups.
//
// Memory traffic per cell: 4 bytes of cost read (sequential 256-byte rows per
// wave) and 1 byte of backtrace code written (8 rows packed per lane into one
// 8-byte store).
#include "common.h"

namespace pardtw {
namespace {

constexpr int kChunk = kBpRows;  // rows per synchronisation chunk (= packed BP group)
constexpr int kRing = 4;         // LDS ring depth, in chunks
constexpr int kPf = 4;           // cost prefetch distance, in chunks
constexpr int kMaxNW = 4;

struct DpShared {
    int super;
    int prog[kMaxNW + 1];  // ring w: chunks published by its producer
    int cons[kMaxNW + 1];  // ring w: chunks released by its consumer
    // ring[w][slot][2e + c] = D[8k - 1 + e][left boundary column c] for chunk k,
    // slot = k % kRing; c = 0 is column 64p-2, c = 1 is column 64p-1.
    float ring[kMaxNW + 1][kRing][2 * kChunk];
};

__device__ inline int lds_get(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_put(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

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
    uint64_t* rec;  // [P][n][2] boundary records
    int64_t n, m;
    int64_t cstride;  // floats between consecutive rows of one panel in C
    int64_t cpanel;   // floats between panels in C (row 0)
    int P;            // number of panels
    int S;            // number of panel groups (= ceil(P / NW))
};

template <int NW>
__device__ void compute_wave(const DpArgs& a, DpShared& sh, int wave, int p, uint32_t epoch) {
    const int lane = threadIdx.x & 63;
    const int64_t n = a.n;
    const int64_t j = int64_t(p) * kPanel + lane;
    const bool colv = j < a.m;
    const int64_t nchunks = ceil_div(n, kChunk);
    const bool have_left = p > 0;
    const bool local_out = (wave < NW - 1) && (p + 1 < a.P);
    const bool global_out = (wave == NW - 1) && (p + 1 < a.P);
    float* rin = &sh.ring[wave][0][0];
    float* rout = &sh.ring[wave + 1][0][0];
    uint64_t* rec_out = a.rec + (size_t(p) * size_t(n)) * 2;
    const int bcol = lane - (kLanes - 2);  // 0/1 on the two boundary lanes
    const bool is_bnd = bcol >= 0;

    const float* cp = a.C + int64_t(p) * a.cpanel + lane;
    const float kInf = __builtin_inff();

    // cost prefetch ring: chunk k lives in cbuf[k % kPf]
    float cbuf[kPf][kChunk];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
#pragma unroll
        for (int r = 0; r < kChunk; ++r) {
            const int64_t i = int64_t(u) * kChunk + r;
            cbuf[u][r] = (colv && i < n) ? __builtin_nontemporal_load(cp + i * a.cstride) : 0.0f;
        }
    }

    float d1 = kInf, s1p = kInf;  // D[i-1][j] and D[i-2][j-1]
    if (local_out && lane >= kLanes - 2) rout[0 * 2 * kChunk + bcol] = kInf;  // row -1 of chunk 0

    for (int64_t k0 = 0; k0 < nchunks; k0 += kPf) {
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            const int64_t k = k0 + u;
            if (k >= nchunks) break;
            const int64_t i0 = k * kChunk;
            const int rows = int(n - i0 < kChunk ? n - i0 : kChunk);
            const int slot = int(k % kRing);

            // left boundary columns for rows i0-1 .. i0+6
            float lv[2 * kChunk];
            if (have_left) {
                while (lds_get(&sh.prog[wave]) <= k) __builtin_amdgcn_s_sleep(1);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
                for (int e = 0; e < 2 * kChunk; ++e) lv[e] = rin[slot * 2 * kChunk + e];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane == 0) lds_put(&sh.cons[wave], int(k + 1));
            } else {
#pragma unroll
                for (int e = 0; e < 2 * kChunk; ++e) lv[e] = kInf;
            }
            // the row i0+7 written below goes to slot k+1: wait until it is free
            if (local_out) {
                while (lds_get(&sh.cons[wave + 1]) < k + 2 - kRing) __builtin_amdgcn_s_sleep(1);
            }

            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int r = 0; r < kChunk; ++r) {
                if (r >= rows) break;
                const int64_t i = i0 + r;
                const float c = cbuf[u][r];
                const float s1 = shift_in(d1, lv[2 * r + 1]);  // D[i-1][j-1]
                const float s2 = shift_in(s1, lv[2 * r]);      // D[i-1][j-2]
                const float c0 = __builtin_fmaf(2.0f, c, s1);
                const float c1 = __builtin_fmaf(3.0f, c, s2);
                const float c2 = __builtin_fmaf(3.0f, c, s1p);
                float best = c0;
                uint32_t code = 0;
                if (c1 < best) { best = c1; code = 1; }
                if (c2 < best) { best = c2; code = 2; }
                if (best == kInf) code = 3;
                if (i == 0 && j == 0) { best = c; code = 3; }
                d1 = best;
                s1p = s1;
                if (r < 4) lo |= code << (8 * r); else hi |= code << (8 * (r - 4));
                if (is_bnd) {
                    if (local_out) {
                        // row i is entry r+1 of chunk k, or entry 0 of chunk k+1
                        const int ds = r + 1 < kChunk ? slot : int((k + 1) % kRing);
                        const int de = r + 1 < kChunk ? r + 1 : 0;
                        rout[(ds * kChunk + de) * 2 + bcol] = best;
                    }
                    if (global_out) {
                        const uint64_t v = (uint64_t(epoch) << 32) | uint64_t(__float_as_uint(best));
                        __hip_atomic_store(rec_out + i * 2 + bcol, v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                if (local_out && r == (rows < kChunk - 1 ? rows - 1 : kChunk - 2)) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    if (lane == 0) lds_put(&sh.prog[wave + 1], int(k + 1));
                }
            }
            uint64_t* bpo = reinterpret_cast<uint64_t*>(a.bp) + ((int64_t(p) * nchunks + k) * kLanes + lane);
            __builtin_nontemporal_store(uint64_t(lo) | (uint64_t(hi) << 32), bpo);

            // refill this buffer with chunk k + kPf
            const int64_t kn = k + kPf;
            if (kn < nchunks) {
#pragma unroll
                for (int r = 0; r < kChunk; ++r) {
                    const int64_t i = kn * kChunk + r;
                    cbuf[u][r] = (colv && i < n) ? __builtin_nontemporal_load(cp + i * a.cstride) : 0.0f;
                }
            }
        }
    }
    if (j == a.m - 1) {
        *a.total = d1;
        *a.status = d1 == kInf ? PARDTW_PAIR_INFEASIBLE : PARDTW_PAIR_OK;
    }
}

// Helper wave: copies the boundary columns of panel pl (the last panel of the
// previous group, computed by another workgroup) from the global records into
// LDS ring 0, chunk by chunk, as soon as their epoch tags show up.
__device__ void helper_wave(const DpArgs& a, DpShared& sh, int pl, uint32_t epoch) {
    const int lane = threadIdx.x & 63;
    const int64_t n = a.n;
    const int64_t nchunks = ceil_div(n, kChunk);
    const uint64_t* rec = a.rec + (size_t(pl) * size_t(n)) * 2;
    float* ring = &sh.ring[0][0][0];
    for (int64_t k = 0; k < nchunks; ++k) {
        const int slot = int(k % kRing);
        while (lds_get(&sh.cons[0]) < k + 1 - kRing) __builtin_amdgcn_s_sleep(1);
        const int64_t row = k * kChunk - 1 + (lane >> 1);
        const bool want = lane < 2 * kChunk && row >= 0 && row < n;
        uint64_t v = 0;
        for (;;) {
            bool ok = true;
            if (want) {
                v = __hip_atomic_load(rec + row * 2 + (lane & 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = uint32_t(v >> 32) == epoch;
            }
            if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
            __builtin_amdgcn_s_sleep(2);
        }
        if (lane < 2 * kChunk) ring[slot * 2 * kChunk + lane] = want ? __uint_as_float(uint32_t(v)) : __builtin_inff();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) lds_put(&sh.prog[0], int(k + 1));
    }
}

template <int NW>
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
            if (p < a.P) compute_wave<NW>(a, sh, wave, p, epoch);
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

}  // namespace

size_t dp_workspace_bytes_impl(int64_t n, int64_t m) {
    return sizeof(DpWsHeader) + size_t(num_panels(m)) * size_t(n) * 2 * sizeof(uint64_t);
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
    a.P = int(num_panels(m));
    if (layout == PARDTW_LAYOUT_PANEL) {
        a.cstride = kPanel;
        a.cpanel = n * kPanel;
    } else {
        a.cstride = m;
        a.cpanel = kPanel;
    }
    const int nw = nw_override > 0 ? nw_override : choose_nw(a.P);
    a.S = int(ceil_div(a.P, nw));
    int dev = 0, cus = 0;
    PARDTW_HIP_TRY(hipGetDevice(&dev));
    PARDTW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = a.S < cus ? a.S : cus;
    dp_prepare<<<1, 1, 0, stream>>>(a.hdr);
    switch (nw) {
        case 1: dp_kernel<1><<<grid, kLanes * 2, 0, stream>>>(a); break;
        case 2: dp_kernel<2><<<grid, kLanes * 3, 0, stream>>>(a); break;
        case 4: dp_kernel<4><<<grid, kLanes * 5, 0, stream>>>(a); break;
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
