// Segment level of Segmental DTW (Sec. II-C steps 3-4; NSDTW's choice, Sec.
// II-B): fragment end columns from the stacked subsequence scores S (row f =
// fragment f, column j = end column).
//
// WSDTW's program Dseg[f,j] = min(Dseg[f,j-1], Dseg[f-1,j-hop] + S[f,j]) is a
// running minimum along each row of t_f[j] = Dseg[f-1,j-hop] + S[f,j], with
// the skip kept on ties, so Dseg[f,j] = min over j' <= j of t_f[j'] and the
// match behind it is the first column where that minimum is reached. Each row
// is therefore one prefix scan of (value, first index) pairs, and row f needs
// only the part of row f-1 that lies hop columns to the left. One workgroup
// owns a row and scans it in tiles of 2048 columns; a tile starts as soon as
// the row above has published the columns it needs, so the rows run as a
// pipeline one tile apart. Values pass between rows as 64-bit records
// {float, uint32 epoch} written and read with agent-scope atomics (the DP's
// boundary handoff), so no side issues a cache-flushing fence. NSDTW is the
// same scan with t_f = S[f, .].
//
// The scan's outputs are Dseg (as records) and, per cell, the first column at
// which the running minimum is reached (int32). The end columns then follow
// from one serial walk over nfrag entries: e_{N-1} = first[N-1][m-1], then
// e_f = first[f][e_{f+1} - hop].
#include "batch.h"

namespace pardtw {
namespace {

constexpr int kSegThreads = 512;
constexpr int kSegPer = 4;                              // columns per thread per tile
constexpr int kSegTile = kSegThreads * kSegPer;         // columns per tile

struct SegHeader {
    uint32_t epoch;
    uint32_t ticket;
    uint32_t pad[62];
};
static_assert(sizeof(SegHeader) == 256, "records stay 256-byte aligned");

struct SegArgs {
    const float* S;
    int64_t nf, m, hop;
    int variant;
    SegHeader* hdr;
    uint64_t* rec;    // [nf][m] Dseg records
    int32_t* first;   // [nf][m] first column of the running minimum (-1 while +inf)
};

// (value, index) running minimum where the earlier element wins ties.
struct VI {
    float v;
    int32_t i;
};
__device__ inline VI later_if_less(VI earlier, VI later) { return later.v < earlier.v ? later : earlier; }

// Lanes of the wave `x` moved by a DPP pattern; lanes that the pattern (or
// the row mask RM) leaves without a source receive the identity (+inf, -1).
template <int CTRL, int RM>
__device__ inline VI dpp_vi(VI x) {
    VI y;
    y.v = __int_as_float(__builtin_amdgcn_update_dpp(int(0x7f800000), __float_as_int(x.v), CTRL, RM, 0xf, false));
    y.i = __builtin_amdgcn_update_dpp(-1, x.i, CTRL, RM, 0xf, false);
    return y;
}

// Inclusive scan of (value, first index) over the 64 lanes: shifts by 1, 2, 4
// and 8 within each row of 16 lanes, then each row takes the total of the rows
// before it (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).
__device__ inline VI wave_scan_vi(VI x) {
    x = later_if_less(dpp_vi<0x111, 0xf>(x), x);
    x = later_if_less(dpp_vi<0x112, 0xf>(x), x);
    x = later_if_less(dpp_vi<0x114, 0xf>(x), x);
    x = later_if_less(dpp_vi<0x118, 0xf>(x), x);
    x = later_if_less(dpp_vi<0x142, 0xa>(x), x);
    x = later_if_less(dpp_vi<0x143, 0xc>(x), x);
    return x;
}

// One workgroup scans a block of up to kSegRows consecutive rows, tile by tile:
// at each tile all rows of the block in order. A row of the block after the
// first reads the row above from LDS, where each row keeps its last two tiles:
// the columns it needs, j - hop for j in the tile, lie in those two tiles when
// hop < kSegTile. The first row of a block reads the row above (the last row
// of the previous block) from its records. So the rows form a chain through
// HBM only once per block. When hop >= kSegTile a block is one row.
constexpr int kSegRows = 8;

__global__ __launch_bounds__(kSegThreads) void segment_scan_kernel(SegArgs a, int rows_per_block) {
    __shared__ VI wave_tot[kSegThreads / 64];
    __shared__ float ring[kSegRows - 1][2][kSegTile];
    __shared__ int ticket;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const uint32_t epoch = __hip_atomic_load(&a.hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float kInf = __builtin_inff();
    const bool wsdtw = a.variant == PARDTW_WSDTW;
    for (;;) {
        __syncthreads();
        if (tid == 0) ticket = int(atomicAdd(&a.hdr->ticket, 1u));
        __syncthreads();
        const int64_t f0 = int64_t(ticket) * rows_per_block;
        if (f0 >= a.nf) break;
        const int rows = int(a.nf - f0 < rows_per_block ? a.nf - f0 : rows_per_block);
        VI carry[kSegRows];
#pragma unroll
        for (int r = 0; r < kSegRows; ++r) carry[r] = VI{kInf, -1};  // running minimum over earlier tiles
        // The scores of every row of the block for one tile, loaded a tile
        // ahead: each row-tile would otherwise wait a memory round trip. The
        // loads are unconditional (rows past the block or the matrix read a
        // valid address, and columns past m are replaced by +inf when used),
        // so the compiler's count of loads in flight stays exact.
        float cb[kSegRows][kSegPer], nb[kSegRows][kSegPer];
        auto load_tile = [&](int64_t tt0, float (&buf)[kSegRows][kSegPer]) {
            const int64_t jj0 = tt0 + int64_t(tid) * kSegPer;
#pragma unroll
            for (int r = 0; r < kSegRows; ++r) {
                const int64_t fr = f0 + r < a.nf ? f0 + r : a.nf - 1;
                const float* srow = a.S + fr * a.m;
#pragma unroll
                for (int e = 0; e < kSegPer; ++e) buf[r][e] = *(jj0 + e < a.m ? srow + jj0 + e : srow);
            }
        };
        load_tile(0, cb);
        int tix = 0;
        for (int64_t t0 = 0; t0 < a.m; t0 += kSegTile, ++tix) {
            const int64_t j0 = t0 + int64_t(tid) * kSegPer;
#pragma unroll
            for (int r = 0; r < kSegRows; ++r) {
                if (r >= rows) break;
                const int64_t f = f0 + r;
                float t[kSegPer];
#pragma unroll
                for (int e = 0; e < kSegPer; ++e) t[e] = (j0 + e < a.m) ? cb[r][e] : kInf;
                if (wsdtw && f > 0) {
                    // Dseg[f-1][j - hop]; +inf left of column hop
                    float pv[kSegPer];
                    if (r == 0) {
                        // the previous block's last row: poll its records until
                        // each needed one carries this launch's epoch
                        const uint64_t* prow = a.rec + (f - 1) * a.m;
                        uint32_t need = 0;
#pragma unroll
                        for (int e = 0; e < kSegPer; ++e) {
                            pv[e] = kInf;
                            if (j0 + e < a.m && j0 + e >= a.hop) need |= 1u << e;
                        }
                        while (need) {
#pragma unroll
                            for (int e = 0; e < kSegPer; ++e) {
                                if (need & (1u << e)) {
                                    const uint64_t v = __hip_atomic_load(prow + (j0 + e - a.hop), __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT);
                                    if (uint32_t(v >> 32) == epoch) {
                                        pv[e] = __uint_as_float(uint32_t(v));
                                        need &= ~(1u << e);
                                    }
                                }
                            }
                            if (need) __builtin_amdgcn_s_sleep(1);
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < kSegPer; ++e) {
                            const int64_t q = j0 + e - a.hop;  // tile tix or tix - 1 (hop < kSegTile)
                            pv[e] = kInf;
                            if (q >= 0 && j0 + e < a.m) {
                                const int qt = int(q / kSegTile);
                                pv[e] = ring[r - 1][qt & 1][int(q - int64_t(qt) * kSegTile)];
                            }
                        }
                    }
#pragma unroll
                    for (int e = 0; e < kSegPer; ++e) t[e] = pv[e] + t[e];
                }
                // the next tile's scores, issued after row 0 has read its
                // records so that the waits of that poll do not cover them
                if (r == 0) load_tile(t0 + kSegTile, nb);
                // this thread's columns
                VI loc[kSegPer];
                VI run{kInf, -1};
#pragma unroll
                for (int e = 0; e < kSegPer; ++e) {
                    run = later_if_less(run, VI{t[e], int32_t(j0 + e)});
                    loc[e] = run;
                }
                // exclusive scan over the wave's lanes (wave_shr:1 of the
                // inclusive one; lane 0 gets the identity)
                const VI inc = wave_scan_vi(run);
                const VI before = dpp_vi<0x138, 0xf>(inc);
                if (lane == 63) wave_tot[wave] = inc;
                __syncthreads();
                VI pre = carry[0];
#pragma unroll
                for (int q = 1; q < kSegRows; ++q) pre = (q == r) ? carry[q] : pre;
                const VI carried = pre;
                for (int w = 0; w < wave; ++w) pre = later_if_less(pre, wave_tot[w]);
                pre = later_if_less(pre, before);
                // the block's last row feeds the next block through records;
                // every row records its last column (the totals)
                const bool last_row = r == rows - 1;
                uint64_t* orow = a.rec + f * a.m;
                int32_t* frow = a.first + f * a.m;
#pragma unroll
                for (int e = 0; e < kSegPer; ++e) {
                    const int64_t j = j0 + e;
                    if (j < a.m) {
                        const VI v = later_if_less(pre, loc[e]);
                        frow[j] = v.i;
                        if (last_row || j == a.m - 1)
                            __hip_atomic_store(orow + j, (uint64_t(epoch) << 32) | uint64_t(__float_as_uint(v.v)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (!last_row) ring[r][tix & 1][int(j - t0)] = v.v;
                    }
                }
                VI nc = carried;
                for (int w = 0; w < kSegThreads / 64; ++w) nc = later_if_less(nc, wave_tot[w]);
#pragma unroll
                for (int q = 0; q < kSegRows; ++q) carry[q] = (q == r) ? nc : carry[q];
                __syncthreads();  // wave_tot and this row's ring tile are read next
            }
#pragma unroll
            for (int r = 0; r < kSegRows; ++r)
#pragma unroll
                for (int e = 0; e < kSegPer; ++e) cb[r][e] = nb[r][e];
        }
    }
}

__global__ void segment_prepare(SegHeader* hdr) {
    hdr->epoch = hdr->epoch + 1;
    hdr->ticket = 0;
}

// One lane walks the fragment ends back from the last one.
__global__ void segment_ends_kernel(SegArgs a, int32_t* ends, float* total, int32_t* status) {
    if (threadIdx.x != 0) return;
    const float kInf = __builtin_inff();
    float tot = 0.0f;
    bool ok = true;
    if (a.variant == PARDTW_WSDTW) {
        tot = __uint_as_float(uint32_t(a.rec[(a.nf - 1) * a.m + a.m - 1]));
        ok = tot < kInf;
        int64_t j = a.m - 1;
        for (int64_t f = a.nf - 1; f >= 0 && ok; --f) {
            const int32_t e = j >= 0 ? a.first[f * a.m + j] : -1;
            if (e < 0) ok = false;
            ends[f] = e;
            j = int64_t(e) - a.hop;
        }
    } else {
        for (int64_t f = 0; f < a.nf; ++f) {
            const int32_t e = a.first[f * a.m + a.m - 1];
            ends[f] = e;
            tot += __uint_as_float(uint32_t(a.rec[f * a.m + a.m - 1]));
            if (e < 0) ok = false;
        }
        ok = ok && tot < kInf;
    }
    if (!ok) {
        for (int64_t f = 0; f < a.nf; ++f) ends[f] = -1;
        tot = kInf;
    }
    *total = tot;
    *status = ok ? PARDTW_PAIR_OK : PARDTW_PAIR_INFEASIBLE;
}

// Concatenation of the fragment paths (each in its own slot of n_f pairs at
// path_off, rows local to the fragment): block f copies fragment f to the sum
// of the lengths before it, shifting rows by the fragment's first row.
__global__ __launch_bounds__(256) void segment_gather_kernel(const BatchPair* __restrict__ pairs, int32_t nf,
                                                             const int32_t* __restrict__ slots,
                                                             const int32_t* __restrict__ frag_len,
                                                             const int32_t* __restrict__ status, int32_t* path,
                                                             int32_t* path_len) {
    __shared__ int64_t base;
    const int f = blockIdx.x;
    const bool ok = *status == PARDTW_PAIR_OK;
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int g = 0; g < f; ++g) s += frag_len[g];
        base = s;
        if (f == nf - 1) *path_len = ok ? int32_t(s + frag_len[f]) : 0;
    }
    __syncthreads();
    if (!ok) return;
    const BatchPair q = pairs[f];
    const int64_t len = frag_len[f];
    const int2* src = reinterpret_cast<const int2*>(slots) + q.path_off;
    int2* dst = reinterpret_cast<int2*>(path) + base;
    for (int64_t c = threadIdx.x; c < len; c += blockDim.x) {
        int2 v = src[c];
        v.x += int32_t(q.x_off);
        dst[c] = v;
    }
}

// Rows of fragments that no end column can be reached for: +inf scores.
__global__ void segment_init_kernel(const BatchPair* __restrict__ pairs, int32_t nf, float* scores,
                                    int32_t* frag_status) {
    const int f = blockIdx.x;
    const BatchPair q = pairs[f];
    if (q.feasible) return;
    for (int64_t j = threadIdx.x; j < q.m; j += blockDim.x) scores[int64_t(f) * q.m + j] = __builtin_inff();
    if (threadIdx.x == 0) frag_status[f] = PARDTW_PAIR_INFEASIBLE;
}

}  // namespace

size_t segment_workspace_bytes_impl(int64_t nf, int64_t m) {
    return sizeof(SegHeader) + size_t(nf) * size_t(m) * (sizeof(uint64_t) + sizeof(int32_t));
}

pardtw_status segment_ends_launch(const float* S, int64_t nf, int64_t m, int64_t hop, int variant, void* ws,
                                  int32_t* ends, float* total, int32_t* status, hipStream_t stream) {
    SegArgs a;
    a.S = S;
    a.nf = nf;
    a.m = m;
    a.hop = hop;
    a.variant = variant;
    a.hdr = reinterpret_cast<SegHeader*>(ws);
    a.rec = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(ws) + sizeof(SegHeader));
    a.first = reinterpret_cast<int32_t*>(a.rec + nf * m);
    int dev = 0, cus = 0;
    PARDTW_HIP_TRY(hipGetDevice(&dev));
    PARDTW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    segment_prepare<<<1, 1, 0, stream>>>(a.hdr);
    // Rows of a block hand over through LDS while the previous row's needed
    // columns lie in its last two tiles; NSDTW rows are independent. A block
    // of R rows makes the chain nf/R handoffs long (about 8 us each) but does
    // tiles x R row-tiles one after another (about 2 us each): R near
    // sqrt(nf * 8 / (2 * tiles)) balances the two (8 at 1000 rows of 100000
    // columns, 2 at 32 rows).
    int rows_per_block = 1;
    if (variant != PARDTW_WSDTW) {
        rows_per_block = kSegRows;
    } else if (hop < kSegTile) {
        const double tiles = double(ceil_div(m, kSegTile));
        const int r = int(__builtin_sqrt(double(nf) * 4.0 / tiles) + 0.5);
        rows_per_block = r < 1 ? 1 : r > kSegRows ? kSegRows : r;
    }
    const int64_t blocks = ceil_div(nf, rows_per_block);
    const int64_t grid2 = blocks < 2 * int64_t(cus) ? blocks : 2 * int64_t(cus);
    segment_scan_kernel<<<unsigned(grid2), kSegThreads, 0, stream>>>(a, rows_per_block);
    segment_ends_kernel<<<1, 64, 0, stream>>>(a, ends, total, status);
    return launch_status();
}

pardtw_status segment_gather_launch(const BatchPair* pairs, int32_t nf, const int32_t* slots,
                                    const int32_t* frag_len, const int32_t* status, int32_t* path,
                                    int32_t* path_len, hipStream_t stream) {
    segment_gather_kernel<<<unsigned(nf), 256, 0, stream>>>(pairs, nf, slots, frag_len, status, path, path_len);
    return launch_status();
}

pardtw_status segment_init_launch(const BatchPair* pairs, int32_t nf, float* scores, int32_t* frag_status,
                                  hipStream_t stream) {
    segment_init_kernel<<<unsigned(nf), 256, 0, stream>>>(pairs, nf, scores, frag_status);
    return launch_status();
}

}  // namespace pardtw

extern "C" size_t pardtw_segment_workspace_bytes(int64_t nfrag, int64_t m) {
    if (nfrag <= 0 || !pardtw::valid_sizes(nfrag, m)) return 0;
    return pardtw::segment_workspace_bytes_impl(nfrag, m);
}

extern "C" pardtw_status pardtw_segment_ends(const float* scores, int64_t nfrag, int64_t m, int64_t hop,
                                             int32_t variant, void* workspace, size_t workspace_bytes,
                                             int32_t* ends, float* total, int32_t* status, hipStream_t stream) {
    if (!scores || !ends || !total || !status || !pardtw::valid_sizes(nfrag, m) || hop < 1)
        return PARDTW_ERR_INVALID_ARG;
    if (nfrag > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    if (variant != PARDTW_NSDTW && variant != PARDTW_WSDTW) return PARDTW_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < pardtw::segment_workspace_bytes_impl(nfrag, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::segment_ends_launch(scores, nfrag, m, hop, variant, workspace, ends, total, status, stream);
}
