// a4: backtrace of the optimal path (Sec. II-D keeps the full backtrace
// matrix; the path is recovered from (N-1, M-1) once the sweep is done).
//
// A walk is serial, so it is built for latency on one workgroup:
//
// * Loaders (waves 1..L). Every step moves 1-2 rows and 1-2 columns, so
//   from a cell (i, j) the path's cells in a column panel p satisfy
//   ceil(dj/2) <= di <= 2 dj, which bounds the rows it can touch there. When
//   the walker enters panel q it asks for panel q - (S - 1); a loader
//   copies exactly those rows' 8-row groups (contiguous in the DP's backtrace
//   layout) into a ring of S LDS slots (slot = panel mod S), compacting the
//   codes to 2 bits on the way: a slot holds one 16-bit word per (group,
//   column) with row r of the group in bits 2r..2r+1. Loader w serves every
//   L-th request, so several requests are in flight at once. (S, L) is (8, 7)
//   for a whole path, (4, 3) for a segment of the split walk below.
// * Walker (wave 0). From the current cell (i, j), lane b holds column j - b
//   and the codes of rows i-31..i in two registers (row i - a in bits
//   30-2a..31-2a of the first for a < 16, of the second as a - 16 otherwise),
//   read with five 16-bit LDS loads. Every step moves at least one column, so
//   a column holds at most one cell of the path, and within 32 rows a path
//   moves at most 62 columns: it leaves the window through the last row. Each
//   lane turns its codes into row masks (rows whose step goes to the next
//   column on the next row, to the next column two rows down, or two columns
//   over on the next row) and the path is traced as a one-cell frontier moved
//   by shifts of those masks and two lane shifts (DPP) per step, all lanes at
//   once. The lane holding a path cell writes it; its index along the path is
//   the number of lower lanes holding one. Near the first row or column a
//   scalar loop checks every step for the origin instead.
// * The path is written from the back of the output (the walk runs backward)
//   and shifted to the front by the whole workgroup at the end.
//
// A subsequence path (Sec. II-B) is walked the same way from (n-1, end) and
// stops on row 0, wherever it lands there.
#include "batch.h"
#include "split.h"
#include "trace.h"

namespace pardtw {
namespace {

// A walker's LDS ring: NS column panels (a power of two) of NG 8-row groups
// each, filled by NL loader waves.
template <int NS, int NG, int NL>
struct WalkShape {
    static constexpr int kS = NS, kG = NG, kL = NL;
    static constexpr int kBytes = NG * kPanel * 2;  // 2-bit codes of one slot
    static constexpr int kThr = kLanes * (1 + NL);
};
// The whole path on one workgroup: panels 7 ahead (at most 101 groups each), 128 KB.
using WalkFull = WalkShape<8, 128, 7>;
// A segment of the split walk: panels 3 ahead (at most 65 groups each), 35 KB,
// so that four segment workgroups share a CU.
using WalkSeg = WalkShape<4, 68, 3>;
constexpr int kSlots = WalkFull::kS;
constexpr int kGroupBytes = kLanes * kBpRows;          // 512 bytes per group in the DP's layout
constexpr int kThreads = WalkFull::kThr;
constexpr int kUnitBytes = kLanes * 16;      // one 16-byte load per lane: 1 KB = two groups
constexpr int kBatch = 16;                   // units in flight per loader wave

template <class W>
struct BtSharedT {
    uint8_t slot[W::kS][W::kBytes];
    int req_panel[W::kS];   // request ring (request r in entry r % kS)
    int req_glo[W::kS];
    int req_ng[W::kS];
    int slot_glo[W::kS];    // first group held by each slot
    int req_count;           // requests issued by the walker
    int loaded[W::kS];      // requests completed per slot
    int done;                // walker finished
    int len;                 // cells on the path (0 on failure)
};
using BtShared = BtSharedT<WalkFull>;

__device__ inline int lds_load_acquire(int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_store_release(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Rows of panel p that a path from (i, j) can touch, as 8-row groups (at most
// NG of them).
template <int NG>
__device__ inline void panel_groups(int i, int j, int p, int& glo, int& ng) {
    const int djmax = j - p * kPanel;
    const int djmin = max(0, j - (p * kPanel + kPanel - 1));
    // clamped at row 0: from a cell the step set cannot reach (only on corrupt
    // codes) the range may be empty, and one group is still requested
    const int rlo = max(0, i - 2 * djmax);
    const int rhi = max(0, i - (djmin + 1) / 2);
    glo = rlo / kBpRows;
    // at most 101 groups for a panel 7 panels ahead, 65 for 3 ahead
    ng = min(rhi / kBpRows - glo + 1, NG);
}

// Eight 2-bit codes (one byte each, values 0..3) to 16 bits.
__device__ inline uint32_t compact8(uint32_t lo, uint32_t hi) {
    uint32_t x = lo & 0x03030303u, y = hi & 0x03030303u;
    x = (x | (x >> 6)) & 0x000F000Fu;
    y = (y | (y >> 6)) & 0x000F000Fu;
    x = (x | (x >> 12)) & 0xFFu;
    y = (y | (y >> 12)) & 0xFFu;
    return x | (y << 8);
}


// Walker: from (i0, j0) back to the origin, or with `sub` to row 0. Returns
// the number of cells written (0 if the codes do not lead there). The output
// holds `cap` pairs; without SEG the k-th cell is written at cap - 1 - k (so
// the path ends up in forward order at the back).
// SEG (one segment of a split walk): the k-th cell is written at k, and with
// stop_row >= 0 the walk ends at the first cell on a row <= stop_row, which is
// not written but returned in *exit; such a walk must stay at row >= 33 and
// column >= 66 (the path's cells there do), else it fails.
template <bool SEG, class W>
__device__ int walk(BtSharedT<W>& sh, int i0, int j0, bool sub, int cap, int32_t* path, int stop_row = -1,
                    int2* exit = nullptr) {
    constexpr int kSlots = W::kS;
    constexpr int kSlotBytes = W::kBytes;
    constexpr int kSlotGroups = W::kG;
    const int lane = threadIdx.x;
    const int P = j0 / kPanel + 1;  // panels the walk can visit
    int i = i0, j = j0, len = 0;
    int nreq = 0;
    auto request = [&](int p) {
        int glo, ng;
        panel_groups<kSlotGroups>(i, j, p, glo, ng);
        const int e = nreq % kSlots;
        if (lane == 0) {
            sh.req_panel[e] = p;
            sh.req_glo[e] = glo;
            sh.req_ng[e] = ng;
            sh.slot_glo[p % kSlots] = glo;
        }
        ++nreq;
        if (lane == 0) lds_store_release(&sh.req_count, nreq);
    };
    auto wait_panel = [&](int p) {
        const int target = ((P - 1 - p) / kSlots) + 1;
        while (lds_load_acquire(&sh.loaded[p % kSlots]) < target) __builtin_amdgcn_s_sleep(1);
        return sh.slot_glo[p % kSlots];
    };
    // On entering panel q the ring holds q .. q-(kSlots-2) and receives
    // q-(kSlots-1); the start enters panel P-1.
    for (int k = 0; k < kSlots && P - 1 - k >= 0; ++k) request(P - 1 - k);
    int cur_q = P - 1;
    int glo0 = wait_panel(cur_q), glo1 = 0;
    bool have1 = false;  // panel cur_q - 1 checked ready

    const uint8_t* lds = &sh.slot[0][0];
    for (;;) {
        if (SEG && i <= stop_row) {
            *exit = make_int2(i, j);
            return len;
        }
        const int q0 = j / kPanel;
        if (q0 != cur_q) {  // entered panel q0 (panels are entered in decreasing order)
            cur_q = q0;
            if (q0 - (kSlots - 1) >= 0) request(q0 - (kSlots - 1));
            glo0 = have1 ? glo1 : wait_panel(q0);
            have1 = false;
        }
        if (!have1 && q0 > 0 && j - (kLanes - 1) < q0 * kPanel) {
            glo1 = wait_panel(q0 - 1);
            have1 = true;
        }

        // lane b: column j - b, rows i-31..i from the five groups from gr on
        uint32_t packed0, packed1;
        {
            const int col = j - lane;
            const int p = col >> 6;  // q0 or q0 - 1 (negative columns give junk)
            const int glo = p == q0 ? glo0 : glo1;
            const uint8_t* base = lds + (p & (kSlots - 1)) * kSlotBytes + (col & (kPanel - 1)) * 2;
            const int gr = (i - 31) >> 3;  // floor, may be negative near row 0
            uint32_t w[5];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                const int lg = min(max(gr + t - glo, 0), kSlotGroups - 1);  // junk outside the slot
                w[t] = *reinterpret_cast<const uint16_t*>(base + lg * (kPanel * 2));
            }
            // row r is at bits 2(r - 8 gr) of w0 | w1 << 16 | ... ; s = i - 8 gr is in [31, 38]
            const int s2 = 2 * (i - 8 * gr);
            const uint64_t lo = uint64_t(w[0]) | (uint64_t(w[1]) << 16) | (uint64_t(w[2]) << 32) | (uint64_t(w[3]) << 48);
            const uint64_t hi = uint64_t(w[1]) | (uint64_t(w[2]) << 16) | (uint64_t(w[3]) << 32) | (uint64_t(w[4]) << 48);
            packed0 = uint32_t(hi >> (s2 - 46));  // rows i .. i-15
            packed1 = uint32_t(lo >> (s2 - 62));  // rows i-16 .. i-31
        }

        if (i >= 33 && j >= 66) {
            // no cell of the window can be the origin or lie outside the matrix
            const WindowMasks wm = window_masks(packed0, packed1);
            // rows above the stop row (bit 31 - a for row a), where the trace may step
            const int above = i - stop_row;
            const uint32_t live = SEG && stop_row >= 0 && above < 32 ? ~(0xFFFFFFFFu >> above) : ~0u;
            const uint32_t on = SEG ? trace_window_live(wm, live, lane) : trace_window(wm, lane);
            if (__builtin_amdgcn_ballot_w64((on & live & wm.two_cols & wm.two_rows) != 0)) return 0;  // code 3
            if constexpr (SEG) {
                // the trace ends on the first cell past the stop row: the last one it marks
                const uint64_t past = __builtin_amdgcn_ballot_w64((on & ~live) != 0);
                if (past) {
                    const int xl = 63 - __builtin_clzll(past);
                    const uint64_t in = past ^ __builtin_amdgcn_ballot_w64(on != 0);
                    const int cnt = __builtin_popcountll(in);
                    if (len + cnt > cap) return 0;
                    if ((on & live) != 0) {
                        const uint32_t lo = uint32_t(in), hi = uint32_t(in >> 32);
                        const int idx = int(__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u)));
                        path[2 * (len + idx)] = i - __builtin_clz(on);
                        path[2 * (len + idx) + 1] = j - lane;
                    }
                    *exit = make_int2(i - __builtin_clz(__builtin_amdgcn_readlane(on, xl)), j - xl);
                    return len + cnt;
                }
            }
            const uint64_t has = __builtin_amdgcn_ballot_w64(on != 0);
            const int cnt = __builtin_popcountll(has);
            const int last = 63 - __builtin_clzll(has);  // lane 0 always holds the start cell
            const uint32_t lm = __builtin_amdgcn_readlane(on, last);
            const int la = __builtin_clz(lm);
            const int a = la + 1 + int((__builtin_amdgcn_readlane(wm.two_rows, last) >> (31 - la)) & 1u);
            const int b = last + 1 + int((__builtin_amdgcn_readlane(wm.two_cols, last) >> (31 - la)) & 1u);
            if (a < 32 || len + cnt > cap) return 0;  // the trace did not leave the window
            if (on != 0) {
                const uint32_t lo = uint32_t(has), hi = uint32_t(has >> 32);
                const int idx = int(__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u)));
                const int64_t pos = SEG ? int64_t(len + idx) : int64_t(cap) - 1 - (len + idx);
                path[2 * pos] = i - __builtin_clz(on);
                path[2 * pos + 1] = j - lane;
            }
            len += cnt;
            i -= a;
            j -= b;
            continue;
        }

        // Near the first row or column: one 16-row half, every step checked
        // (uniform scalar loop). Bit 1 of a code says the step takes two rows,
        // bit 0 two columns, so the unused code 3 reads as an illegal (2, 2)
        // step and is caught after the loop.
        if (SEG && stop_row >= 0) return 0;
        int off = 30, b = 0, k0 = 0;
        uint64_t codes0 = 0;
        bool origin = false;
        int a;
        const int ij = i + j;
        for (;;) {
            a = (30 - off) >> 1;
            if (sub ? a == i : a + b == ij) { origin = true; break; }  // a <= i and b <= j here
            const uint32_t w = __builtin_amdgcn_readlane(packed0, b);
            const uint32_t c = (w >> off) & 3u;
            codes0 |= uint64_t(c) << (2 * k0);
            ++k0;
            off -= 2 + int(c & 2u);
            b += 1 + int(c & 1u);
            if ((30 - off) >> 1 > i || b > j) return 0;  // left the matrix
            if (off < 0) { a = (30 - off) >> 1; break; }
        }
        if ((codes0 & (codes0 >> 1)) & 0x5555555555555555ull) return 0;  // code 3
        const int cnt = k0 + (origin ? 1 : 0);
        if (len + cnt > cap) return 0;
        if (lane < cnt) {
            // offsets after the first `lane` steps
            const uint64_t m0 = (uint64_t(1) << (2 * lane)) - 1;
            const int da = lane + __builtin_popcountll(codes0 & m0 & 0xAAAAAAAAAAAAAAAAull);
            const int db = lane + __builtin_popcountll(codes0 & m0 & 0x5555555555555555ull);
            const int64_t pos = SEG ? int64_t(len + lane) : int64_t(cap) - 1 - (len + lane);
            path[2 * pos] = i - da;
            path[2 * pos + 1] = j - db;
        }
        len += cnt;
        if (origin) return len;
        i -= a;
        j -= b;
    }
}

// Loader wave w: serves requests w, w + kLoaders, ... (each alone), compacting
// the codes of each (group, column) to 16 bits. With PACK the codes already are
// 16 bits per (group, column) in HBM, in the slot's own order, so the
// requested groups are copied as they are.
template <bool PACK, class W>
__device__ void load_panels(BtSharedT<W>& sh, const uint8_t* bp, int64_t G, int w) {
    constexpr int kSlots = W::kS;
    const int lane = threadIdx.x & (kLanes - 1);
    for (int r = w;; r += W::kL) {
        while (lds_load_acquire(&sh.req_count) <= r) {
            if (lds_load_acquire(&sh.done)) return;
            __builtin_amdgcn_s_sleep(2);
        }
        const int e = r % kSlots;
        const int p = sh.req_panel[e];
        const int glo = sh.req_glo[e];
        if constexpr (PACK) {
            const int bytes = sh.req_ng[e] * kPanel * 2;  // a multiple of 128
            const uint8_t* src = bp + (int64_t(p) * G + glo) * (kPanel * 2);
            uint8_t* dst = sh.slot[p % kSlots];
            for (int u0 = 0; u0 < bytes; u0 += kUnitBytes * kBatch) {
                uint4 buf[kBatch];
#pragma unroll
                for (int t = 0; t < kBatch; ++t) {
                    const int off = u0 + t * kUnitBytes + lane * 16;
                    buf[t] = *reinterpret_cast<const uint4*>(src + (off < bytes ? off : bytes - 16));
                }
#pragma unroll
                for (int t = 0; t < kBatch; ++t) {
                    const int off = u0 + t * kUnitBytes + lane * 16;
                    if (off < bytes) *reinterpret_cast<uint4*>(dst + off) = buf[t];
                }
            }
            if (lane == 0)
                __hip_atomic_fetch_add(&sh.loaded[p % kSlots], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            continue;
        }
        const int bytes = sh.req_ng[e] * kGroupBytes;
        const int units = (bytes + kUnitBytes - 1) / kUnitBytes;
        const uint8_t* src = bp + (int64_t(p) * G + glo) * kGroupBytes;
        uint8_t* dst = sh.slot[p % kSlots];
        for (int u0 = 0; u0 < units; u0 += kBatch) {
            uint4 buf[kBatch];
#pragma unroll
            for (int t = 0; t < kBatch; ++t) {
                const int off = (u0 + t) * kUnitBytes + lane * 16;
                const int offc = off < bytes ? off : bytes - 16;  // stays inside the requested groups
                buf[t] = *reinterpret_cast<const uint4*>(src + offc);
            }
#pragma unroll
            for (int t = 0; t < kBatch; ++t) {
                const int off = (u0 + t) * kUnitBytes + lane * 16;
                if (off < bytes) {
                    // 16 bytes = columns c, c+1 of group lg, 8 codes each
                    const int lg = off / kGroupBytes;
                    const int c = (off % kGroupBytes) / kBpRows;
                    const uint32_t pair = compact8(buf[t].x, buf[t].y) | (compact8(buf[t].z, buf[t].w) << 16);
                    *reinterpret_cast<uint32_t*>(dst + lg * (kPanel * 2) + c * 2) = pair;
                }
            }
        }
        if (lane == 0) __hip_atomic_fetch_add(&sh.loaded[p % kSlots], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Moves path entries [base, base + len) to [0, len) in place: each batch is
// read completely before it is written, and later batches read only entries
// at or above the ones this batch writes.
__device__ void shift_path(int32_t* path, int64_t base, int64_t len) {
    constexpr int kPer = 8;
    int2* pp = reinterpret_cast<int2*>(path);
    for (int64_t q0 = 0; q0 < len; q0 += int64_t(kThreads) * kPer) {
        int2 v[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int64_t q = q0 + t * kThreads + threadIdx.x;
            if (q < len) v[t] = pp[base + q];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int64_t q = q0 + t * kThreads + threadIdx.x;
            if (q < len) pp[q] = v[t];
        }
        __syncthreads();
    }
}

// One path: DTW from (n-1, m-1) when `ok` (the pair's status), or with `sub`
// from (n-1, j_end) to row 0. PACK: codes packed 2 bits per cell.
template <bool PACK = false>
__device__ void backtrace_pair(BtShared& sh, const uint8_t* bp, int n, int j_end, bool sub, bool ok, int cap,
                               int32_t* path, int32_t* path_len) {
    const int tid = threadIdx.x;
    if (!ok) {
        if (tid == 0) *path_len = 0;
        return;
    }
    if (tid < kSlots) sh.loaded[tid] = 0;
    if (tid == 0) {
        sh.req_count = 0;
        sh.done = 0;
        sh.len = 0;
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wave == 0) {
        const int len = walk<false>(sh, n - 1, j_end, sub, cap, path);
        if (tid == 0) {
            sh.len = len;
            lds_store_release(&sh.done, 1);
        }
    } else {
        load_panels<PACK>(sh, bp, bp_groups(n), wave - 1);
    }
    __syncthreads();
    const int len = sh.len;
    __threadfence_block();
    shift_path(path, int64_t(cap) - len, len);
    if (tid == 0) *path_len = len;
}

// A subsequence end is usable when it is a column of the matrix that row 0
// reaches at row n-1.
__device__ inline bool sub_end_ok(int64_t n, int64_t m, int32_t e) { return e >= 0 && e < m && 2 * int64_t(e) >= n - 1; }

// ---- Split walk (split.h) ----------------------------------------------------
// The segments are walked by the walker above with a stop row, on the smaller
// ring of WalkSeg.
struct SegArgs : SplitArgs {
    const uint8_t* bp;
};

using SegShared = BtSharedT<WalkSeg>;

// One segment walk by the whole workgroup (walker wave 0, loader waves
// 1..L); the record goes to info_out and, for every thread, to `res`.
template <bool PACK>
__device__ SegInfo walk_segment(SegShared& sh, SegInfo& res, const SegArgs& a, int s, int si, int sj,
                                SegInfo* info_out) {
    const int tid = threadIdx.x;
    if (tid < WalkSeg::kS) sh.loaded[tid] = 0;
    if (tid == 0) {
        sh.req_count = 0;
        sh.done = 0;
        sh.len = 0;
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wave == 0) {
        int2 ex = make_int2(-1, -1);
        const int len = walk<true>(sh, si, sj, a.sub != 0, a.R, a.cells + int64_t(s) * a.R * 2, seg_stop_row(s, a.R),
                                   &ex);
        if (tid == 0) {
            const SegInfo r = seg_info(si, sj, ex.x, ex.y, len);
            *info_out = r;
            res = r;
            lds_store_release(&sh.done, 1);
        }
    } else {
        load_panels<PACK>(sh, a.bp, bp_groups(a.n), wave - 1);
    }
    __syncthreads();
    return res;
}

template <bool PACK>
__device__ void seg_round_body(SegShared& sh, SegInfo& res, const SegArgs& a, int s, int round) {
    split_round(a, s, round, [&](int s_, int si, int sj, SegInfo* out) {
        return walk_segment<PACK>(sh, res, a, s_, si, sj, out);
    });
}

template <bool PACK>
__device__ void seg_finish_body(SegShared& sh, SegInfo& res, SegInfo* sinfo, const SegArgs& a, int fin, int cap,
                                int32_t* path_len) {
    split_finish(a, sinfo, fin, cap, path_len, [&](int s_, int si, int sj, SegInfo* out) {
        return walk_segment<PACK>(sh, res, a, s_, si, sj, out);
    });
}

__device__ void seg_copy_body(const SegArgs& a, int s, int fin, int32_t* path) { split_copy(a, s, fin, path); }

// One pair: workgroup s walks segment s.
template <bool PACK>
__global__ __launch_bounds__(WalkSeg::kThr) void seg_round_kernel(SegArgs a, const int32_t* __restrict__ status,
                                                                   int round) {
    __shared__ SegShared sh;
    __shared__ SegInfo res;
    if (*status != PARDTW_PAIR_OK) return;
    seg_round_body<PACK>(sh, res, a, blockIdx.x, round);
}

template <bool PACK>
__global__ __launch_bounds__(WalkSeg::kThr) void seg_finish_kernel(SegArgs a, const int32_t* __restrict__ status,
                                                                    int fin, int cap, int32_t* path_len) {
    __shared__ SegShared sh;
    __shared__ SegInfo res;
    __shared__ SegInfo sinfo[kSegMaxCount];
    if (*status != PARDTW_PAIR_OK) {
        if (threadIdx.x == 0) *path_len = 0;
        return;
    }
    seg_finish_body<PACK>(sh, res, sinfo, a, fin, cap, path_len);
}

__global__ __launch_bounds__(256) void seg_copy_kernel(SegArgs a, int fin, const int32_t* __restrict__ path_len,
                                                       int32_t* __restrict__ path) {
    if (*path_len <= 0) return;
    seg_copy_body(a, blockIdx.x, fin, path);
}

// Batched form: the pairs listed in `sp` are split (segment g belongs to
// sp[seg_map[g]]); the others keep the one-workgroup walk. With `ends` the
// pairs are the fragments of a Segmental DTW plan, walked as subsequence
// paths from (n-1, ends[pair]); otherwise DTW pairs with their `status`.
struct SegBatchArgs {
    const BatchPair* pairs;
    const SegPair* sp;
    const int32_t* seg_map;
    const uint8_t* bp;     // codes of the batch
    const int32_t* status;
    const int32_t* ends;
    SegInfo* info;         // the split region: SegInfo entries, then cells
    int32_t* cells;
    int32_t* paths;
    int32_t* path_len;
};

__device__ inline SegArgs seg_args_of(const SegBatchArgs& ba, const SegPair& sp) {
    const BatchPair q = ba.pairs[sp.pair];
    SegArgs a;
    a.bp = ba.bp + q.bp_off;
    a.n = int(q.n);
    a.m = int(q.m);
    a.end = ba.ends ? ba.ends[sp.pair] : int(q.m - 1);
    a.sub = ba.ends ? 1 : 0;
    a.R = sp.R;
    a.S = sp.S;
    a.info = ba.info + sp.info_off;
    a.cells = ba.cells + sp.cells_off;
    return a;
}

// Whether the pair has a path to walk: a DTW pair's status, a fragment's end.
__device__ inline bool seg_pair_ok(const SegBatchArgs& ba, const SegPair& sp) {
    if (!ba.ends) return ba.status[sp.pair] == PARDTW_PAIR_OK;
    const BatchPair q = ba.pairs[sp.pair];
    return q.feasible && sub_end_ok(q.n, q.m, ba.ends[sp.pair]);
}

__global__ __launch_bounds__(WalkSeg::kThr) void seg_round_batch_kernel(SegBatchArgs ba, int round) {
    __shared__ SegShared sh;
    __shared__ SegInfo res;
    const SegPair sp = ba.sp[ba.seg_map[blockIdx.x]];
    if (!seg_pair_ok(ba, sp)) return;
    seg_round_body<false>(sh, res, seg_args_of(ba, sp), int(blockIdx.x) - sp.seg0, round);
}

__global__ __launch_bounds__(WalkSeg::kThr) void seg_finish_batch_kernel(SegBatchArgs ba, int fin) {
    __shared__ SegShared sh;
    __shared__ SegInfo res;
    __shared__ SegInfo sinfo[kSegMaxCount];
    const SegPair sp = ba.sp[blockIdx.x];
    int32_t* plen = ba.path_len + sp.pair;
    if (!seg_pair_ok(ba, sp)) {
        if (threadIdx.x == 0) *plen = 0;
        return;
    }
    const BatchPair q = ba.pairs[sp.pair];
    // a subsequence path has one cell per row at most, a DTW path min(n, m)
    const int cap = ba.ends ? int(q.n) : int(q.n < q.m ? q.n : q.m);
    seg_finish_body<false>(sh, res, sinfo, seg_args_of(ba, sp), fin, cap, plen);
}

__global__ __launch_bounds__(256) void seg_copy_batch_kernel(SegBatchArgs ba, int fin) {
    const SegPair sp = ba.sp[ba.seg_map[blockIdx.x]];
    if (ba.path_len[sp.pair] <= 0) return;
    seg_copy_body(seg_args_of(ba, sp), int(blockIdx.x) - sp.seg0, fin, ba.paths + 2 * ba.pairs[sp.pair].path_off);
}

__global__ __launch_bounds__(kThreads) void backtrace_kernel(const uint8_t* __restrict__ bp, int64_t n, int64_t m,
                                                             const int32_t* __restrict__ status, int32_t* path,
                                                             int32_t* path_len) {
    __shared__ BtShared sh;
    backtrace_pair(sh, bp, int(n), int(m - 1), false, *status == PARDTW_PAIR_OK, int(n < m ? n : m), path, path_len);
}

__global__ __launch_bounds__(kThreads) void backtrace_packed_kernel(const uint8_t* __restrict__ bp2, int64_t n,
                                                                    int64_t m, const int32_t* __restrict__ status,
                                                                    int32_t* path, int32_t* path_len) {
    __shared__ BtShared sh;
    backtrace_pair<true>(sh, bp2, int(n), int(m - 1), false, *status == PARDTW_PAIR_OK, int(n < m ? n : m), path,
                         path_len);
}

__global__ __launch_bounds__(kThreads) void subseq_backtrace_kernel(const uint8_t* __restrict__ bp, int64_t n,
                                                                    int64_t m, const int32_t* __restrict__ end_col,
                                                                    int32_t* path, int32_t* path_len) {
    __shared__ BtShared sh;
    const int32_t e = *end_col;
    backtrace_pair(sh, bp, int(n), e, true, sub_end_ok(n, m, e), int(n), path, path_len);
}

// Fragments of a Segmental DTW plan: workgroup b walks fragment b from ends[b]
// into its own slot of n_b pairs.
__global__ __launch_bounds__(kThreads) void subseq_backtrace_batch_kernel(const BatchPair* __restrict__ pairs,
                                                                          const uint8_t* __restrict__ bpbase,
                                                                          const int32_t* __restrict__ ends,
                                                                          int32_t* paths, int32_t* path_len) {
    __shared__ BtShared sh;
    const int b = blockIdx.x;
    const BatchPair q = pairs[b];
    if (q.split) return;  // walked by the split kernels
    const int32_t e = ends[b];
    backtrace_pair(sh, bpbase + q.bp_off, int(q.n), e, true, q.feasible && sub_end_ok(q.n, q.m, e), int(q.n),
                   paths + 2 * q.path_off, path_len + b);
}

// Batched form: workgroup b walks pair b (infeasible pairs just get length 0).
__global__ __launch_bounds__(kThreads) void backtrace_batch_kernel(const BatchPair* __restrict__ pairs,
                                                                   const uint8_t* __restrict__ bpbase,
                                                                   const int32_t* __restrict__ status,
                                                                   int32_t* paths, int32_t* path_len) {
    __shared__ BtShared sh;
    const int b = blockIdx.x;
    const BatchPair q = pairs[b];
    if (q.split) return;  // walked by the split kernels
    const bool ok = q.feasible && status[b] == PARDTW_PAIR_OK;
    backtrace_pair(sh, bpbase + q.bp_off, int(q.n), int(q.m - 1), false, ok, int(q.n < q.m ? q.n : q.m),
                   paths + 2 * q.path_off, path_len + b);
}

__global__ void bp_unpack_kernel(const uint8_t* __restrict__ bp, int64_t n, int64_t m, int8_t* __restrict__ out) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t i = idx / m, j = idx % m;
    out[idx] = int8_t(bp[bp_offset(n, i, j)]);
}

__global__ void bp2_unpack_kernel(const uint16_t* __restrict__ bp2, int64_t n, int64_t m, int8_t* __restrict__ out) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t i = idx / m, j = idx % m;
    const int64_t word = (j / kPanel * bp_groups(n) + i / kBpRows) * kPanel + j % kPanel;
    out[idx] = int8_t((bp2[word] >> (2 * (i % kBpRows))) & 3u);
}

}  // namespace

pardtw_status backtrace_batch_launch(const BatchPair* pairs, int32_t batch, const uint8_t* bpbase,
                                     const int32_t* status, int32_t* paths, int32_t* path_len, hipStream_t stream) {
    if (batch <= 0) return PARDTW_OK;
    backtrace_batch_kernel<<<unsigned(batch), kThreads, 0, stream>>>(pairs, bpbase, status, paths, path_len);
    return launch_status();
}

pardtw_status subseq_backtrace_batch_launch(const BatchPair* pairs, int32_t batch, const uint8_t* bpbase,
                                            const int32_t* ends, int32_t* paths, int32_t* path_len,
                                            hipStream_t stream) {
    if (batch <= 0) return PARDTW_OK;
    subseq_backtrace_batch_kernel<<<unsigned(batch), kThreads, 0, stream>>>(pairs, bpbase, ends, paths, path_len);
    return launch_status();
}

}  // namespace pardtw

extern "C" pardtw_status pardtw_backtrace(const uint8_t* bp, int64_t n, int64_t m, const int32_t* pair_status,
                                          int32_t* path, int32_t* path_len, hipStream_t stream) {
    if (!bp || !pair_status || !path || !path_len || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(path) % 8 != 0) return PARDTW_ERR_INVALID_ARG;
    pardtw::backtrace_kernel<<<1, pardtw::kThreads, 0, stream>>>(bp, n, m, pair_status, path, path_len);
    return pardtw::launch_status();
}

namespace pardtw {
namespace {

constexpr int kSegMinRows = 512;  // rows per segment at least
constexpr int kSegMax = kSegMaxCount;
constexpr int kSegRounds = 3;     // parallel rounds before the check

void seg_shape(int64_t n, int& R, int& S) {
    const int64_t r = ceil_div(n, int64_t(kSegMax));
    R = int(r > kSegMinRows ? r : kSegMinRows);
    S = int(ceil_div(n, int64_t(R)));
}

size_t seg_bytes(int64_t n) {
    int R, S;
    seg_shape(n, R, S);
    return size_t(2) * S * sizeof(SegInfo) + size_t(S) * R * 2 * sizeof(int32_t);
}

template <bool PACK>
pardtw_status seg_backtrace(const uint8_t* bp, int64_t n, int64_t m, const int32_t* status, int32_t* path,
                            int32_t* path_len, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!bp || !status || !path || !path_len || !ws || !valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(path) % 8 != 0 || reinterpret_cast<uintptr_t>(ws) % 16 != 0)
        return PARDTW_ERR_INVALID_ARG;
    if (PACK && reinterpret_cast<uintptr_t>(bp) % 16 != 0) return PARDTW_ERR_INVALID_ARG;
    if (ws_bytes < seg_bytes(n)) return PARDTW_ERR_WORKSPACE;
    SegArgs a;
    a.bp = bp;
    a.n = int(n);
    a.m = int(m);
    a.end = int(m - 1);
    a.sub = 0;
    seg_shape(n, a.R, a.S);
    if (a.S <= 2) {
        // a pair of at most 1024 rows: one workgroup walks it faster than
        // five launches split it
        if (PACK) backtrace_packed_kernel<<<1, kThreads, 0, stream>>>(bp, n, m, status, path, path_len);
        else backtrace_kernel<<<1, kThreads, 0, stream>>>(bp, n, m, status, path, path_len);
        return launch_status();
    }
    a.info = reinterpret_cast<SegInfo*>(ws);
    a.cells = reinterpret_cast<int32_t*>(a.info + 2 * a.S);
    for (int r = 0; r < kSegRounds; ++r) seg_round_kernel<PACK><<<a.S, WalkSeg::kThr, 0, stream>>>(a, status, r);
    const int fin = (kSegRounds - 1) & 1;
    seg_finish_kernel<PACK><<<1, WalkSeg::kThr, 0, stream>>>(a, status, fin, int(n < m ? n : m), path_len);
    seg_copy_kernel<<<a.S, 256, 0, stream>>>(a, fin, path_len, path);
    return launch_status();
}

}  // namespace

void split_shape(int64_t n, int& R, int& S) { seg_shape(n, R, S); }

size_t split_record_bytes() { return sizeof(SegInfo); }

pardtw_status split_backtrace_batch_launch(const BatchPair* pairs, const SegPair* sp, int32_t nsplit,
                                           const int32_t* seg_map, int32_t nseg, const uint8_t* bpbase,
                                           const int32_t* status, const int32_t* ends, void* records,
                                           int32_t* cells, int32_t* paths, int32_t* path_len, hipStream_t stream) {
    if (nsplit <= 0 || nseg <= 0) return PARDTW_OK;
    SegBatchArgs ba;
    ba.pairs = pairs;
    ba.sp = sp;
    ba.seg_map = seg_map;
    ba.bp = bpbase;
    ba.status = status;
    ba.ends = ends;
    ba.info = reinterpret_cast<SegInfo*>(records);
    ba.cells = cells;
    ba.paths = paths;
    ba.path_len = path_len;
    for (int r = 0; r < kSegRounds; ++r) seg_round_batch_kernel<<<nseg, WalkSeg::kThr, 0, stream>>>(ba, r);
    const int fin = (kSegRounds - 1) & 1;
    seg_finish_batch_kernel<<<nsplit, WalkSeg::kThr, 0, stream>>>(ba, fin);
    seg_copy_batch_kernel<<<nseg, 256, 0, stream>>>(ba, fin);
    return launch_status();
}

}  // namespace pardtw

extern "C" size_t pardtw_backtrace_parallel_bytes(int64_t n, int64_t m) {
    if (!pardtw::valid_sizes(n, m)) return 0;
    return pardtw::seg_bytes(n);
}

extern "C" pardtw_status pardtw_backtrace_parallel(const uint8_t* bp, int64_t n, int64_t m,
                                                   const int32_t* pair_status, int32_t* path, int32_t* path_len,
                                                   void* workspace, size_t workspace_bytes, hipStream_t stream) {
    return pardtw::seg_backtrace<false>(bp, n, m, pair_status, path, path_len, workspace, workspace_bytes, stream);
}

extern "C" pardtw_status pardtw_backtrace_packed_parallel(const uint16_t* bp2, int64_t n, int64_t m,
                                                          const int32_t* pair_status, int32_t* path,
                                                          int32_t* path_len, void* workspace,
                                                          size_t workspace_bytes, hipStream_t stream) {
    return pardtw::seg_backtrace<true>(reinterpret_cast<const uint8_t*>(bp2), n, m, pair_status, path, path_len,
                                       workspace, workspace_bytes, stream);
}

extern "C" pardtw_status pardtw_subseq_backtrace(const uint8_t* bp, int64_t n, int64_t m, const int32_t* end_col,
                                                 int32_t* path, int32_t* path_len, hipStream_t stream) {
    if (!bp || !end_col || !path || !path_len || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(path) % 8 != 0) return PARDTW_ERR_INVALID_ARG;
    pardtw::subseq_backtrace_kernel<<<1, pardtw::kThreads, 0, stream>>>(bp, n, m, end_col, path, path_len);
    return pardtw::launch_status();
}

extern "C" pardtw_status pardtw_bp_unpack(const uint8_t* bp, int64_t n, int64_t m, int8_t* out, hipStream_t stream) {
    if (!bp || !out || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    const int64_t cells = n * m;
    const int64_t blocks = pardtw::ceil_div(cells, 256);
    if (blocks > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    pardtw::bp_unpack_kernel<<<unsigned(blocks), 256, 0, stream>>>(bp, n, m, out);
    return pardtw::launch_status();
}

extern "C" pardtw_status pardtw_backtrace_packed(const uint16_t* bp2, int64_t n, int64_t m,
                                                 const int32_t* pair_status, int32_t* path, int32_t* path_len,
                                                 hipStream_t stream) {
    if (!bp2 || !pair_status || !path || !path_len || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(path) % 8 != 0 || reinterpret_cast<uintptr_t>(bp2) % 16 != 0)
        return PARDTW_ERR_INVALID_ARG;
    pardtw::backtrace_packed_kernel<<<1, pardtw::kThreads, 0, stream>>>(reinterpret_cast<const uint8_t*>(bp2), n, m,
                                                                       pair_status, path, path_len);
    return pardtw::launch_status();
}

extern "C" pardtw_status pardtw_bp2_unpack(const uint16_t* bp2, int64_t n, int64_t m, int8_t* out,
                                           hipStream_t stream) {
    if (!bp2 || !out || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    const int64_t blocks = pardtw::ceil_div(n * m, 256);
    if (blocks > 0x7fffffff) return PARDTW_ERR_UNSUPPORTED;
    pardtw::bp2_unpack_kernel<<<unsigned(blocks), 256, 0, stream>>>(bp2, n, m, out);
    return pardtw::launch_status();
}
