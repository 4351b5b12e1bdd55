// a3: the ParDTW accumulated-cost dynamic program on gfx950.
//
// Recurrence (Sec. V step set {(1,1),(1,2),(2,1)}, weights {2,3,3}):
//   D[i,j] = min(D[i-1,j-1] + 2C, D[i-1,j-2] + 3C, D[i-2,j-1] + 3C),  D[0,0] = C[0,0].
// The same sweep runs subsequence DTW (Sec. II-B, the frame-level step of
// Segmental DTW): weights {1,1,2}, every cell of row 0 a start, D[0,j] = C[0,j],
// and the last row D[n-1, .] as output.
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
// Panel p starts chunk k (8 rows) once panel p-1 has published chunk k, so
// the sweep front is a staircase along the anti-diagonal of the (row, panel)
// grid and every panel is active at once.
//
// A workgroup holds NW compute waves (NW consecutive panels) and two helper
// waves. Boundary columns pass between the compute waves of a workgroup through
// LDS rings, 8 rows at a time; between workgroups the output helper forwards
// the last wave's ring to global records {float D, uint32 epoch} written with
// agent-scope 64-bit atomic stores, which the input helper of the next
// workgroup polls, several chunks per round trip, into its first ring, so no
// side issues a cache-flushing fence. A pair's boundaries take record columns
// round robin from kRecSlots of them, one column of n rows each: at most
// `grid` groups run at once and a group's input helper ends before the next
// group's, so while group q runs every boundary below q - grid has been read
// (the tags carry the column's lap parity besides the launch epoch). Records
// then take 16 B per row and resident workgroup, not per row and panel. The first panel's ring is filled with
// +inf once. Every compute wave thus runs the same instructions each chunk:
// only its waits depend on its role, and no register value does, which keeps
// the compiler from copying the boundary registers and from waiting on their
// LDS reads early. Workgroups take groups
// of panels from an atomic ticket in increasing order; a group only waits on
// lower tickets, held by running workgroups, so the sweep always makes
// progress whatever the number of resident workgroups.
//
// Memory traffic per cell: 4 bytes of cost read and 1 byte of backtrace code
// written. In the panel layout a wave reads a chunk's 2 KB of cost with two
// loads of 1 KB contiguous each (16 bytes per lane) and writes its 512 bytes
// of codes with one store (8 bytes per lane).
//
// Fused cost (the paper computes costs inside the DP, Sec. II-D): each compute
// wave gets a producer wave that computes its panel's costs from the features,
// 16 rows at a time with the cost GEMM's own MFMA slab (cost_slab.h), into an
// LDS ring the compute wave reads instead of HBM. The DP then moves 1 byte per
// cell (the codes) and its costs are bit for bit those of the GEMM.
#include <mutex>
#include <type_traits>

#include "batch.h"
#include "cost_slab.h"
#include "dp_step.h"

// Workspace of pardtw_dp_noalloc: one array per GPU for the life of the
// process, zero at load like every device global without an initialiser.
// Host code must not pass this name to a kernel (on the host it is only a
// stand-in for the symbol): its device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[PARDTW_NOALLOC_SCRATCH_BYTES];

namespace pardtw {
namespace {

constexpr int kRing = 32;        // LDS ring depth, in chunks
constexpr int kPfPanel = 4;      // cost prefetch distance in chunks, panel layout (4 measured best of 2-16)
constexpr int kPfRow = 4;        // the same for the row-major layout (8 loads per chunk)
constexpr int kHelperWin = 4;   // chunks polled per helper round trip (one record per lane)
constexpr int kMaxNWFused = 4;   // fused workgroups: NW compute + NW producer + 2 helper waves
constexpr int kCRing = 8;        // fused cost ring depth, in chunks (2 KB each)
constexpr int kPfFused = 4;      // fused cost chunks read ahead of the one computed
// the consumer releases ring slots once per group of kPfFused chunks, kPfFused
// chunks behind its reads, and the producer writes two chunks at a time
static_assert(kCRing >= kPfFused + 2, "fused cost ring too shallow for the read-ahead");
constexpr int kRecSlots = 257;   // record columns of one pair; the grid stays below it

// Where the DP's costs come from.
// kSrcFusedCk: fused costs, no codes, and D of the last two rows of every
// block of rows saved for the checkpointed backtrace.
// kSrcPanelPk / kSrcFusedPk: panel or fused costs, codes packed 2 bits per
// cell (one 16-bit word per column and 8-row group).
// kSrcFusedB: fused costs from BF16 operands (d <= 128, d % 8 == 0), those of
// the cost GEMM's BF16 sweep; at most two compute waves per workgroup.
enum CostSrc { kSrcRow = 0, kSrcPanel = 1, kSrcFused = 2, kSrcFusedCk = 3, kSrcPanelPk = 4, kSrcFusedPk = 5,
               kSrcFusedB = 6 };
constexpr bool is_fused(int src) {
    return src == kSrcFused || src == kSrcFusedCk || src == kSrcFusedPk || src == kSrcFusedB;
}
constexpr int kMaxNWFusedB = 2;  // BF16 producers hold about 230 registers: two waves per SIMD
constexpr bool is_packed(int src) { return src == kSrcPanelPk || src == kSrcFusedPk; }

// Fused cost: per compute wave a ring of cost chunks in the panel layout
// (rows 0-3 of the 64 columns, then rows 4-7), and its progress counters.
struct CostRing {
    float slot[kMaxNWFused][kCRing][kChunk * kLanes];
    int prog[kMaxNWFused];  // chunks whose costs are in the ring (or need none)
    int cons[kMaxNWFused];  // chunks the compute wave has taken out
};

template <int NW>
struct DpShared {
    int super;
    int prog[NW + 1][2];  // ring w: chunks published by its producer (two copies, see below)
    int cons[NW + 1];  // ring w: chunks released by its consumer
    // ring[w][slot][c][r] = D[8k + r][64p - 2 + c] for chunk k, slot = k % kRing
    float ring[NW + 1][kRing][2][kChunk];
    // Lanes that have nothing to hand over write here instead, so the handoff
    // stores run on the full wave without masking the execution mask.
    f32x4 fsink[NW][kLanes][2];
    int isink[NW][kLanes];
};

struct DpArgs {
    const float* C;
    const float* X;  // fused cost: features (n x d, m x d FP32, d <= 16)
    const float* Y;
    const float* rxs;  // fused cost: inverse norms of the rows of X, zero padded
    int64_t d;
    uint8_t* bp;
    float* total;   // DTW: D[n-1][m-1]; subsequence DTW: the m scores D[n-1][.]
    int32_t* status;
    DpWsHeader* hdr;
    // Boundary records, [column][G*8][2] {float D, uint32 tag}. rec_slots > 0:
    // boundary q (group q to q + 1) in column q % rec_slots; rec_slots == 0:
    // one column per panel, boundary q in column q*NW + NW - 1.
    uint64_t* rec;
    int rec_slots;
    int64_t n, m;
    int64_t G;      // 8-row groups per panel
    int P;          // number of panels
    int S;          // number of panel groups (= ceil(P / NW))
    // kSrcFusedCk: D of rows (q+1)K-2 and (q+1)K-1 for q < ck_count, stored at
    // ckpt[(2q + t) * ck_stride + column], K = 8 * ck_chunks
    float* ckpt;
    int ck_chunks;
    int ck_count;
    int64_t ck_stride;
};

// Loads chunk k of panel p into cb. Every call issues the same loads: when
// `real` is false (a chunk whose result is known without its costs, or one
// past the end) the loads read the panel's first chunk instead, which stays
// cached; each panel uses its own, so these reads spread over the caches. Unconditional loads keep the compiler's count of outstanding
// memory operations exact, so the prefetch ring really stays kPf chunks deep.
template <int SRC>
__device__ __attribute__((always_inline)) inline void load_chunk(const DpArgs& a, int p, int lane, int k, bool real,
                                                                 float (&cb)[kChunk]) {
    if constexpr (SRC != kSrcRow) {
        // rows 0-3 of the chunk for all 64 columns, then rows 4-7: each load
        // instruction reads 1 KB of contiguous memory
        // a chunk whose costs are not needed reads panel 0's first chunk,
        // which holds the origin and so is always written (finite costs)
        const float* base = real ? a.C + (int64_t(p) * a.G + k) * (kLanes * kChunk) : a.C;
        const f32x4* src = reinterpret_cast<const f32x4*>(base) + lane;
        const f32x4 v0 = __builtin_nontemporal_load(src);
        const f32x4 v1 = __builtin_nontemporal_load(src + kLanes);
        cb[0] = v0[0]; cb[1] = v0[1]; cb[2] = v0[2]; cb[3] = v0[3];
        cb[4] = v1[0]; cb[5] = v1[1]; cb[6] = v1[2]; cb[7] = v1[3];
    } else {
        // padding lanes and rows read element 0; their results are never used
        const int64_t j = int64_t(p) * kPanel + lane;
        const bool colv = j < a.m;
#pragma unroll
        for (int r = 0; r < kChunk; ++r) {
            const int64_t i = int64_t(k) * kChunk + r;
            const int64_t off = (real && colv && i < a.n) ? i * a.m + j : 0;
            cb[r] = __builtin_nontemporal_load(a.C + off);
        }
    }
}

// Loads the panel-layout cost chunk at base into cb (see load_chunk).
__device__ __attribute__((always_inline)) inline void load_chunk_at(const float* base, int lane, float (&cb)[kChunk]) {
    const f32x4* src = reinterpret_cast<const f32x4*>(base) + lane;
    const f32x4 v0 = __builtin_nontemporal_load(src);
    const f32x4 v1 = __builtin_nontemporal_load(src + kLanes);
    cb[0] = v0[0]; cb[1] = v0[1]; cb[2] = v0[2]; cb[3] = v0[3];
    cb[4] = v1[0]; cb[5] = v1[1]; cb[6] = v1[2]; cb[7] = v1[3];
}

// Chunks whose costs the sweep reads: those of the band of cells that can lie
// on a path from (0,0) to (N-1,M-1). Every other chunk runs the same
// instructions on a cost chunk that is always written (the origin's), so the
// loop has one path, and its values do not matter:
// * a cell unreachable from the origin has only unreachable predecessors, so
//   its D stays +inf whatever the finite costs;
// * a cell that cannot reach the end feeds only cells that cannot either, so
//   whatever finite D it gets never reaches a band cell.
// Band cells are thus exact and, being reachable, finite: they need no
// unreachable test, and the codes of cells outside the band are unspecified.
struct ChunkRanges {
    int lo, hi;  // [lo, hi], empty when lo > hi
};

// Subsequence DTW uses its own band (a path starts anywhere on row 0 and ends
// anywhere on row n-1); the same two arguments hold for it.
template <bool SUB>
__device__ inline ChunkRanges chunk_ranges(int p, int64_t n, int64_t m, int64_t G) {
    ChunkRanges r;
    const int64_t lo = SUB ? sub_group_lo(p, n, m) : band_group_lo(p, n, m);
    const int64_t hi = SUB ? sub_group_hi(p, n, m) : band_group_hi(p, n, m);
    r.lo = int(lo < G ? lo : G);
    r.hi = int(hi < G - 1 ? hi : G - 1);
    return r;
}

// The first chunk a panel reads from its left neighbour: the chunk above its
// first band chunk when the left panel computes it (its rows feed the first
// band row), else the first band chunk itself. Panel 0 reads its +inf source.
template <bool SUB>
__device__ inline int first_input_chunk(int p, int64_t n, int64_t m, int64_t G) {
    const int k0 = chunk_ranges<SUB>(p, n, m, G).lo;
    if (p == 0 || k0 == 0) return k0;
    const int kl = chunk_ranges<SUB>(p - 1, n, m, G).lo;
    return k0 - 1 >= kl ? k0 - 1 : k0;
}

// A compute wave owns panel p. Whether it feeds a right neighbour is a runtime
// value made opaque to the optimiser and only gates a rare wait, so every role
// runs the same instructions: the unrolled chunk loop is large and several
// roles sharing one instruction cache would otherwise evict each other.
// Chunk k's costs from the fused ring into cb, once the producer has them
// (chunks past the end read a slot without waiting; their values are unused).
__device__ __attribute__((always_inline)) inline void ring_chunk(CostRing& cr, int wave, int lane, int k, int klast,
                                                                 int& cprog_seen, float (&cb)[kChunk],
                                                                 bool release = true) {
    if (k <= klast)
        while (cprog_seen <= k) cprog_seen = lds_get(&cr.prog[wave]);
    compiler_order();
    const f32x4* src = reinterpret_cast<const f32x4*>(&cr.slot[wave][unsigned(k) % unsigned(kCRing)][0]) + lane;
    const f32x4 v0 = src[0], v1 = src[kLanes];
    cb[0] = v0[0]; cb[1] = v0[1]; cb[2] = v0[2]; cb[3] = v0[3];
    cb[4] = v1[0]; cb[5] = v1[1]; cb[6] = v1[2]; cb[7] = v1[3];
    compiler_order();
    // the slot is free once read (LDS operations of a wave complete in order)
    if (release) lds_put(&cr.cons[wave], k + 1);
}

template <int SRC, bool SUB, class Sh>
__device__ __attribute__((always_inline)) inline void compute_wave(const DpArgs& a, Sh& sh, CostRing* cring,
                                                                   int wave, int p, bool have_out) {
    const int lane = threadIdx.x & 63;
    const int G = int(a.G);  // chunks per panel (rows padded to a multiple of 8)
    // The panel sweeps only its band chunks k0 .. k1 (Section "ChunkRanges").
    const ChunkRanges cr = chunk_ranges<SUB>(p, a.n, a.m, a.G);
    const int k0 = cr.lo, k1 = cr.hi;
    // The left panel publishes its chunks from its own first band chunk on;
    // row 8 k0 - 1 and 8 k0 - 2 of it (chunk k0 - 1) feed this panel's first
    // band row when they are band chunks of the left panel, else +inf does.
    const int kin = first_input_chunk<SUB>(p, a.n, a.m, a.G);
    // Chunks k1 + 1 .. khr of the right panel's band get +inf boundary columns.
    const int khr = have_out ? chunk_ranges<SUB>(p + 1, a.n, a.m, a.G).hi : k1;
    const float kInf = __builtin_inff();
    const int bcol = lane - (kLanes - 2);  // 0 / 1 on the two boundary lanes
    uint64_t* bp_pan = reinterpret_cast<uint64_t*>(a.bp) + int64_t(p) * G * kLanes;
    // the code store of chunk k0, advanced one chunk per chunk (8 bytes per
    // lane, or 2 with packed codes)
    uint64_t* cptr = is_packed(SRC) ? reinterpret_cast<uint64_t*>(reinterpret_cast<uint16_t*>(a.bp) +
                                                                   (int64_t(p) * G + k0) * kLanes)
                                    : bp_pan + int64_t(k0) * kLanes;
    const float* rin = &sh.ring[wave][0][0][0];
    float* rout = &sh.ring[wave + 1][0][0][0];
    // a boundary lane's column in the output ring (slot 0); other lanes write
    // to their sink
    float* wbase = bcol >= 0 ? rout + bcol * kChunk : reinterpret_cast<float*>(&sh.fsink[wave][lane][0]);
    int flags = __builtin_amdgcn_readfirstlane(have_out ? 2 : 0);
    // chunks before kin are never read: release their ring slots at once
    if (lane == 0) lds_put(&sh.cons[wave], kin);

    constexpr bool kFused = is_fused(SRC);
    constexpr bool kCk = SRC == kSrcFusedCk;
    // the first chunk at or after k0 that ends a block of rows, and its checkpoint
    int ck_q = kCk ? (k0 + 1 + a.ck_chunks - 1) / a.ck_chunks - 1 : 0;
    int ck_next = kCk ? (ck_q + 1) * a.ck_chunks - 1 : 0;
    const int ck_q0 = ck_q;
    constexpr bool kPack = is_packed(SRC);
    constexpr int kPf = kFused ? kPfFused : SRC == kSrcRow ? kPfRow : kPfPanel;
    float cbuf[kPf][kChunk];
    int cprog_seen = 0, cpv = 0;
    if constexpr (kFused) {
        if (lane == 0) lds_put(&cring->cons[wave], k0);
#pragma unroll
        for (int u = 0; u < kPf; ++u) ring_chunk(*cring, wave, lane, k0 + u, k1, cprog_seen, cbuf[u]);
    } else {
#pragma unroll
        for (int u = 0; u < kPf; ++u)
            load_chunk<SRC>(a, p, lane, k0 + u, k0 + u <= k1, cbuf[u]);
    }
    // panel layouts: the chunk kPf ahead, advanced one chunk per chunk
    const float* cnext = a.C + (int64_t(p) * G + k0 + kPf) * (kLanes * kChunk);

    // Rows above the first band chunk: D of this panel's own columns there
    // is +inf (no band cell has a finite predecessor there), and lane 0
    // takes the left panel's rows 8 k0 - 1 and 8 k0 - 2 from its chunk k0 - 1.
    float e0 = kInf, e1 = kInf, s1p0 = kInf;
    int prog_seen = 0, pv = 0;
    if (kin < k0) {
        while (prog_seen <= kin) prog_seen = lds_get(&sh.prog[wave][0]);
        compiler_order();
        const float* src = rin + (kin % kRing) * 2 * kChunk;
        e0 = src[kChunk - 1];
        e1 = src[2 * kChunk - 1];
        s1p0 = src[2 * kChunk - 2];
        compiler_order();
        if (lane == 0) lds_put(&sh.cons[wave], k0);
    }
    // D[i-1][j] and D[i-2][j-1]. The origin is produced by the general rule
    // through a virtual D[-2][-1] = -2 C[0][0]: fma(3, C00, -2 C00) = C00
    // exactly, and that value is used by no other cell. Subsequence DTW starts
    // on every cell of row 0 the same way: fma(2, C0j, -C0j) = C0j.
    float d1 = kInf;
    float s1p = lane == 0 ? s1p0 : kInf;
    if (k0 == 0) s1p = SUB ? -cbuf[0][0] : (p == 0 && lane == 0) ? -2.0f * cbuf[0][0] : s1p;
    const int last = G - 1;
    const int rlast = int((a.n - 1) % kChunk);
    float dlast = kInf;
    int cons_seen = 0;

    // Boundary columns of chunk k: a consumer starts chunk k as soon as its
    // producer has published chunk k. Row 0 of a chunk needs only the last
    // boundary row of the chunk before (e0, e1), so the LDS reads of chunk k's
    // boundary are in flight while row 0 is computed. The producer's progress
    // counter is read asynchronously one chunk before it is tested.
    float lv0[kChunk], lv1[kChunk];

    // The unrolled body has no early exit: chunks past k1 (at most kPf - 1)
    // run as known chunks whose code store goes to a sink and whose boundary
    // goes to a ring nobody reads. Every path then issues the same memory
    // operations, which keeps the compiler's outstanding-load counts exact
    // across the loop back edge.
    // The chunks go in groups of kPf. whole: 0 any group; 1 band chunks only,
    // so the tests of `inside` fold away; 2 band chunks whose prefetches (kPf
    // ahead) are band chunks too. Groups 1 and 2 also check the right ring's
    // space and release their input slots once per group instead of once per
    // chunk. A wave issues one instruction at a time and the sweep's chain
    // runs through every chunk, so each instruction taken out of a chunk
    // shortens the sweep: this took the DP from 3.38 to 2.79 ms.
    auto group = [&](int kb, auto whole) {
        if constexpr (decltype(whole)::value >= 1) {
            if ((flags & 2) && cons_seen < kb + kPf - kRing) {
                int v;
                while ((v = lds_get(&sh.cons[wave + 1])) < kb + kPf - kRing) {}
                cons_seen = v;
            }
        }
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            const int k = kb + u;
            const bool inside = decltype(whole)::value ? true : k <= k1;
            asm volatile("" : "+s"(flags));
            const int slot = int(unsigned(k) % unsigned(kRing));

            {
                // Compute waves own their SIMD, so a consumer that caught up spins
                // on the counter without sleeping: each late wake-up would be
                // lost time it could never win back, adding up along the chain.
                // Only the wait is conditional: the reads below always run, so
                // their registers need no copies and their latency stays hidden.
                if (inside)
                    while (prog_seen <= k) prog_seen = lds_get(&sh.prog[wave][0]);
                compiler_order();
                const f32x4* src = reinterpret_cast<const f32x4*>(rin + slot * 2 * kChunk);
                const f32x4 x0 = src[0], x1 = src[1], y0 = src[2], y1 = src[3];
                lv0[0] = x0[0]; lv0[1] = x0[1]; lv0[2] = x0[2]; lv0[3] = x0[3];
                lv0[4] = x1[0]; lv0[5] = x1[1]; lv0[6] = x1[2]; lv0[7] = x1[3];
                lv1[0] = y0[0]; lv1[1] = y0[1]; lv1[2] = y0[2]; lv1[3] = y0[3];
                lv1[4] = y1[0]; lv1[5] = y1[1]; lv1[6] = y1[2]; lv1[7] = y1[3];
                compiler_order();
                if constexpr (!decltype(whole)::value) lds_put(lane == 0 ? &sh.cons[wave] : &sh.isink[wave][lane], k + 1);
                // read per lane from one of two identical copies, so the value
                // stays in a vector register and is not waited for until the
                // end of the chunk. (The compiler issues the read near its use,
                // at the chunk's end, which sees the left panel's latest
                // progress: pinning it here measured slower, 2.84 against
                // 2.80 ms, as an older value sends more chunks to the spin.)
                pv = lds_get(&sh.prog[wave][lane & 1]);
                // the same for the cost producer's counter
                if constexpr (kFused) cpv = lds_get(&cring->prog[wave]);
            }

            uint32_t lo, hi;
            float best_r[kChunk];
            dp_rows<SUB, kPack>(cbuf[u], lv0, lv1, e0, e1, d1, s1p, lo, hi, best_r);
            if constexpr (!decltype(whole)::value) {
                if (SUB) {
                    if (k == 0) lo = (lo & ~0xffu) | 3u;  // row 0: every cell is a start
                } else if (p == 0 && k == 0 && lane == 0) {
                    const uint32_t row0 = kPack ? 0x3u : 0xffu;
                    lo = (lo & ~row0) | 3u;  // the origin's code
                }
            }
            e0 = lv0[kChunk - 1];
            e1 = lv1[kChunk - 1];

            if constexpr (kCk) {
                // no codes; rows 6 and 7 of a chunk that ends a block are the
                // two rows the block after it starts from
                if (k == ck_next && inside && ck_q < a.ck_count) {
                    float* dst = a.ckpt + int64_t(2 * ck_q) * a.ck_stride + int64_t(p) * kPanel + lane;
                    dst[0] = best_r[kChunk - 2];
                    dst[a.ck_stride] = best_r[kChunk - 1];
                    ++ck_q;
                    ck_next += a.ck_chunks;
                }
            } else if constexpr (kPack) {
                // one 16-bit word per lane: 128 bytes per chunk
                uint16_t* cdst = inside ? reinterpret_cast<uint16_t*>(cptr) : reinterpret_cast<uint16_t*>(a.hdr->sink);
                cptr = reinterpret_cast<uint64_t*>(reinterpret_cast<uint16_t*>(cptr) + kLanes);
                __builtin_nontemporal_store(uint16_t(lo), cdst + lane);
            } else {
                uint64_t* cdst = inside ? cptr : a.hdr->sink;
                cptr += kLanes;
                // as a pair of words: the row step's two words go to the store's
                // registers without the copies a 64-bit OR costs
                typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
                __builtin_nontemporal_store(u32x2{lo, hi}, reinterpret_cast<u32x2*>(cdst + lane));
            }

            // LDS operations complete in issue order. Drain this chunk's reads
            // (issued a whole chunk ago, so already done) before issuing the
            // ring writes below, so that no later wait queues behind fresh writes.
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
            {
                const int pv0 = __builtin_amdgcn_readfirstlane(pv);
                // the counter only grows, and pv was read after every earlier read of it
                prog_seen = pv0;
                if constexpr (kFused) cprog_seen = __builtin_amdgcn_readfirstlane(cpv);
            }

            {
                // A wave without a right neighbour writes into a ring nobody reads.
                if (!decltype(whole)::value && (flags & 2) && inside && cons_seen < k + 1 - kRing) {
                    int v;
                    while ((v = lds_get(&sh.cons[wave + 1])) < k + 1 - kRing) {}
                    cons_seen = v;
                }
                compiler_order();
                {
                    f32x4* dst = (bcol >= 0 && inside) ? reinterpret_cast<f32x4*>(wbase + slot * 2 * kChunk)
                                                       : &sh.fsink[wave][lane][0];
                    dst[0] = f32x4{best_r[0], best_r[1], best_r[2], best_r[3]};
                    dst[1] = f32x4{best_r[4], best_r[5], best_r[6], best_r[7]};
                }
                compiler_order();
                lds_put(lane < 2 ? &sh.prog[wave + 1][lane] : &sh.isink[wave][lane], inside ? k + 1 : k1 + 1);
            }
            if (!decltype(whole)::value && k == last && inside) {
#pragma unroll
                for (int r = 0; r < kChunk; ++r) dlast = (r == rlast) ? best_r[r] : dlast;
            }

            const int kn = k + kPf;
            if constexpr (kFused) ring_chunk(*cring, wave, lane, kn, k1, cprog_seen, cbuf[u], !decltype(whole)::value);
            else if constexpr (SRC == kSrcRow) load_chunk<SRC>(a, p, lane, kn <= k1 ? kn : k0, kn <= k1, cbuf[u]);
            else {
                load_chunk_at(decltype(whole)::value == 2 || kn <= k1 ? cnext : a.C, lane, cbuf[u]);
                cnext += kLanes * kChunk;
            }
        }
        if constexpr (decltype(whole)::value >= 1) {
            compiler_order();
            lds_put(lane == 0 ? &sh.cons[wave] : &sh.isink[wave][lane], kb + kPf);
            // the cost slots of every chunk read so far
            if constexpr (kFused) lds_put(&cring->cons[wave], kb + 2 * kPf);
        }
    };
    // Chunk 0 (the origin, or subsequence DTW's row of starts) and the
    // matrix's last chunk (the total) are left to the general groups.
    int kb = k0;
    if (k0 == 0) {
        group(kb, std::integral_constant<int, 0>{});
        kb += kPf;
    }
    const int kw_end = k1 == last ? k1 - 1 : k1;
    if constexpr (!kFused && SRC != kSrcRow)
        for (; kb + 2 * kPf - 1 <= kw_end; kb += kPf) group(kb, std::integral_constant<int, 2>{});
    for (; kb + kPf - 1 <= kw_end; kb += kPf) group(kb, std::integral_constant<int, 1>{});
    for (; kb <= k1; kb += kPf) group(kb, std::integral_constant<int, 0>{});
    // Chunks k1 + 1 .. khr of the right panel's band: their left boundary lies
    // outside this panel's band, so it is handed over as +inf.
    if (flags & 2) {
        for (int k = k1 + 1; k <= khr; ++k) {
            if (cons_seen < k + 1 - kRing) {
                int v;
                while ((v = lds_get(&sh.cons[wave + 1])) < k + 1 - kRing) {}
                cons_seen = v;
            }
            compiler_order();
            if (bcol >= 0) {
                f32x4* dst = reinterpret_cast<f32x4*>(rout + ((k % kRing) * 2 + bcol) * kChunk);
                dst[0] = f32x4{kInf, kInf, kInf, kInf};
                dst[1] = f32x4{kInf, kInf, kInf, kInf};
            }
            compiler_order();
            if (lane < 2) lds_put(&sh.prog[wave + 1][lane], k + 1);
        }
    }
    if constexpr (kCk) {
        // checkpoints of blocks that end outside the band chunks: +inf
        for (int q = 0; q < a.ck_count; ++q) {
            if (q >= ck_q0 && q < ck_q) continue;
            float* dst = a.ckpt + int64_t(2 * q) * a.ck_stride + int64_t(p) * kPanel + lane;
            dst[0] = kInf;
            dst[a.ck_stride] = kInf;
        }
    }
    // DTW: total = D[n-1][m-1]. Subsequence DTW: the whole last row, whose
    // last column is reachable whenever any is (+inf in panels whose band
    // stops above the last row).
    const int64_t col = int64_t(p) * kPanel + lane;
    if (SUB && col < a.m) a.total[col] = dlast;
    if (col == a.m - 1) {
        if (!SUB) *a.total = dlast;
        *a.status = dlast == kInf ? PARDTW_PAIR_INFEASIBLE : PARDTW_PAIR_OK;
    }
}

// Producer of compute wave w (panel p) in the fused form: the panel's costs,
// 16 rows (two chunks) at a time, into the wave's ring. Only the slabs that
// hold a band chunk are visited; the compute wave reads whatever finite values
// a slot holds for the other chunk of a slab (zeros at first), which only
// reach cells outside the band.
__device__ __attribute__((always_inline)) inline void cost_producer(const DpArgs& a, CostRing& cr, int w, int p,
                                                                    bool sub) {
    const int lane = threadIdx.x & 63;
    const int G = int(a.G);
    // the band's chunks, clamped to the rows (the subsequence bound runs past them)
    const int64_t lo = sub ? sub_group_lo(p, a.n, a.m) : band_group_lo(p, a.n, a.m);
    const int64_t hi_raw = sub ? sub_group_hi(p, a.n, a.m) : band_group_hi(p, a.n, a.m);
    const int64_t hi = hi_raw < G - 1 ? hi_raw : G - 1;
    float bv[4][4], ry[4];
    panel_operands_f32_small(a.Y, a.m, a.d, p, bv, ry);
    f32x4* ring = reinterpret_cast<f32x4*>(&cr.slot[w][0][0]);
    // the lane's four rows of a slab: row0 + 4*(lane/16) + r
    const f32x4* rx_base = reinterpret_cast<const f32x4*>(a.rxs) + (lane >> 4);
    for (int e = lane; e < kCRing * kChunk * kLanes / 4; e += kLanes) ring[e] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int cons_seen = 0;
    // rows 4*(lane/16) + r of the slab: chunk 2s + lane/32, half (lane/16) % 2
    const int kq = lane >> 5, half = (lane >> 4) & 1, col = lane & 15;
    // Row operands and row norms two slabs ahead, in three rotating buffers:
    // step s first issues slab s+2's loads, then computes slab s, whose loads
    // went out two steps earlier with four slabs' worth after them. The loop
    // is unrolled by three (padded with slabs past the end, which compute and
    // write nothing), so every path through it issues the same loads and no
    // register with a load in flight is copied. Rows past n read the zero
    // padding of the row-norm area.
    const float* zeros = a.rxs + a.n;
    if (lo > hi) {
        lds_put(&cr.prog[w], G);
        return;
    }
    const int s0 = int(lo >> 1), s1 = int(hi >> 1);
    float avA[4], avB[4], avC[4];
    f32x4 rxA, rxB, rxC;
    // (issued in slab order, as the loop issues them, so that the compiler's
    // load counts agree on both ways into the loop)
    slab_rows_f32_small_ahead(a.X, zeros, a.n, a.d, int64_t(16) * s0, avA);
    rxA = rx_base[4 * s0];
    compiler_order();
    slab_rows_f32_small_ahead(a.X, zeros, a.n, a.d, int64_t(16) * (s0 + 1), avB);
    rxB = rx_base[4 * (s0 + 1)];
    compiler_order();
    auto step = [&](int s, float (&av)[4], f32x4& rx, float (&av_next)[4], f32x4& rx_next) {
        slab_rows_f32_small_ahead(a.X, zeros, a.n, a.d, int64_t(16) * (s + 2), av_next);
        rx_next = rx_base[4 * (s + 2)];
        const int k0 = 2 * s;
        if (s <= s1) {
            const int need = k0 + 2 - kCRing;  // the consumer has taken chunk k0 + 1 - kCRing out
            while (cons_seen < need) {
                cons_seen = lds_get(&cr.cons[w]);
                if (cons_seen < need) __builtin_amdgcn_s_sleep(1);
            }
            f32x4 acc[4], v[4];
            slab_acc_f32_small(a.d, av, bv, acc);
            costs_from_acc_rx(acc, rx, ry, v);
            const int kk = k0 + kq;
            if (kk < G) {
                float* dst = &cr.slot[w][kk % kCRing][half * (kLanes * 4)];
#pragma unroll
                for (int b = 0; b < 4; ++b) *reinterpret_cast<f32x4*>(dst + (b * 16 + col) * 4) = v[b];
            }
        }
        compiler_order();
        lds_put(&cr.prog[w], k0 + 2 < G ? k0 + 2 : G);
    };
    for (int s = s0; s <= s1; s += 3) {
        step(s, avA, rxA, avC, rxC);
        step(s + 1, avB, rxB, avA, rxA);
        step(s + 2, avC, rxC, avB, rxB);
    }
}

// Producer of compute wave w (panel p) from BF16 operands (d <= 128, d % 8 ==
// 0): the panel operands, row operands, MFMA steps and their order are those
// of the cost GEMM's BF16 sweep (cost_slab.h), so the costs are the same
// bits; the row norms come from the row operands, as there. Only the band's
// slabs are visited. Each step issues the raw row features of the slab two
// ahead into one of three rotating register sets (rows past n read row n-1,
// which is zeroed after the load), then converts and computes its own slab.
__device__ __attribute__((always_inline)) inline void cost_producer_bf16(const DpArgs& a, CostRing& cr, int w,
                                                                         int p, bool sub) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int G = int(a.G);
    // the band's chunks, clamped to the rows (the subsequence bound runs past
    // them): the consumer takes chunks up to G - 1 only, so a slab past them
    // would wait for ring space forever
    const int64_t lo = sub ? sub_group_lo(p, a.n, a.m) : band_group_lo(p, a.n, a.m);
    const int64_t hi_raw = sub ? sub_group_hi(p, a.n, a.m) : band_group_hi(p, a.n, a.m);
    const int64_t hi = hi_raw < G - 1 ? hi_raw : G - 1;
    bf16x8 bv[4][4];
    float ry[4];
    panel_operands_bf16<true>(a.Y, a.m, a.d, p, bv, ry);
    f32x4* ring = reinterpret_cast<f32x4*>(&cr.slot[w][0][0]);
    for (int e = lane; e < kCRing * kChunk * kLanes / 4; e += kLanes) ring[e] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t L = (a.d + 31) / 32 * 8;  // features per lane group
    const int kq = lane >> 5, half = (lane >> 4) & 1, col = lane & 15;
    int cons_seen = 0;
    auto load_rows = [&](int s, f32x4 (&raw)[8]) {
        const int64_t row = int64_t(16) * s + (lane & 15);
        const float* xr = a.X + (row < a.n ? row : a.n - 1) * a.d;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t k0 = g * L + 8 * t;
            const int64_t kc = k0 + 8 <= a.d ? k0 : a.d - 8;  // in the row (d >= 8)
            raw[2 * t] = *reinterpret_cast<const f32x4*>(xr + kc);
            raw[2 * t + 1] = *reinterpret_cast<const f32x4*>(xr + kc + 4);
        }
    };
    auto compute = [&](int s, const f32x4 (&raw)[8], f32x4 (&v)[4]) {
        const bool ok = int64_t(16) * s + (lane & 15) < a.n;
        float sa = 0.0f;
        bf16x8 av[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            av[t] = bf16x8{};
            if (8 * t < L) {
                const bool okk = ok && g * L + 8 * t < a.d;  // d % 8 == 0: all eight or none
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = okk ? raw[2 * t + (e >> 2)][e & 3] : 0.0f;
                av[t] = cvt8_bf16(x, sa);
            }
        }
        f32x4 acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (8 * t < L)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], bv[b][t], acc[b], 0, 0, 0);
        costs_from_acc(acc, inv_from_sq(sum_groups(sa)), ry, v);
    };
    if (lo > hi) {
        lds_put(&cr.prog[w], G);
        return;
    }
    const int s0 = int(lo >> 1), s1 = int(hi >> 1);
    f32x4 rA[8], rB[8], rC[8];
    load_rows(s0, rA);
    compiler_order();
    load_rows(s0 + 1, rB);
    compiler_order();
    auto step = [&](int s, f32x4 (&cur)[8], f32x4 (&nxt)[8]) {
        load_rows(s + 2, nxt);
        const int k0 = 2 * s;
        if (s <= s1) {
            const int need = k0 + 2 - kCRing;  // the consumer has taken chunk k0 + 1 - kCRing out
            while (cons_seen < need) {
                cons_seen = lds_get(&cr.cons[w]);
                if (cons_seen < need) __builtin_amdgcn_s_sleep(1);
            }
            f32x4 v[4];
            compute(s, cur, v);
            const int kk = k0 + kq;
            if (kk < G) {
                float* dst = &cr.slot[w][kk % kCRing][half * (kLanes * 4)];
#pragma unroll
                for (int b = 0; b < 4; ++b) *reinterpret_cast<f32x4*>(dst + (b * 16 + col) * 4) = v[b];
            }
        }
        compiler_order();
        lds_put(&cr.prog[w], k0 + 2 < G ? k0 + 2 : G);
    };
    for (int s = s0; s <= s1; s += 3) {
        step(s, rA, rC);
        step(s + 1, rB, rA);
        step(s + 2, rC, rB);
    }
}

// Input helper: copies the boundary columns of panel pl (the last panel of the
// previous group, computed by another workgroup) from the global records into
// LDS ring 0. One poll reads kHelperWin chunks (16 records each, one per
// lane) and publishes every leading chunk whose epoch tags are all present.
// Polls are back to back: under full memory load a poll's round trip is the
// handoff's latency, and it grows with the loads a poll issues (windows of
// 8, 16 or more chunks measured slower).
template <bool SUB, class Sh>
__device__ __attribute__((always_inline)) inline void in_helper(const DpArgs& a, Sh& sh, int pl,
                                                                const uint64_t* rec, uint32_t tag) {
    constexpr int kPer = kHelperWin * 16 / kLanes;  // records per lane per poll
    const int lane = threadIdx.x & 63;
    const int64_t G = a.G;
    float* ring = &sh.ring[0][0][0][0];
    int cons_seen = 0;
    // the chunks the group's first panel (pl + 1) reads
    const int64_t khi = chunk_ranges<SUB>(pl + 1, a.n, a.m, G).hi;
    for (int64_t k = first_input_chunk<SUB>(pl + 1, a.n, a.m, G); k <= khi;) {
        uint64_t v[kPer];
        uint64_t good[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int e = lane + kLanes * t;  // record within the window
            const int64_t kq = k + (e >> 4);
            bool ok = true;
            v[t] = 0;
            if (kq <= khi) {
                v[t] = __hip_atomic_load(rec + (kq * kChunk + ((e & 15) >> 1)) * 2 + (e & 1), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
                ok = uint32_t(v[t] >> 32) == tag;
            }
            good[t] = __builtin_amdgcn_ballot_w64(ok);
        }
        int ready = 0;
        while (ready < kHelperWin && k + ready <= khi &&
               ((good[ready >> 2] >> (16 * (ready & 3))) & 0xffffull) == 0xffffull)
            ++ready;
        if (ready == 0) continue;
        if (cons_seen < k + ready - kRing) {
            int c;
            while ((c = lds_get(&sh.cons[0])) < k + ready - kRing) __builtin_amdgcn_s_sleep(1);
            cons_seen = c;
        }
        compiler_order();
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int e = lane + kLanes * t;
            if ((e >> 4) < ready) {
                const int64_t kq = k + (e >> 4);
                ring[(int(kq % kRing) * 2 + (e & 1)) * kChunk + ((e & 15) >> 1)] = __uint_as_float(uint32_t(v[t]));
            }
        }
        compiler_order();
        if (lane < 2) lds_put(&sh.prog[0][lane], int(k + ready));
        k += ready;
    }
}

// Input of the first panel: no left neighbour, so every boundary value is
// +inf; the ring is filled once and published as complete.
template <class Sh>
__device__ __attribute__((always_inline)) inline void inf_source(Sh& sh) {
    const int lane = threadIdx.x & 63;
    float* ring = &sh.ring[0][0][0][0];
    for (int e = lane; e < kRing * 2 * kChunk; e += kLanes) ring[e] = __builtin_inff();
    compiler_order();
    if (lane < 2) lds_put(&sh.prog[0][lane], 1 << 30);
}

// Output helper: forwards the boundary columns that the last compute wave of
// the group (panel pl) leaves in LDS ring NW to the global records, up to four
// chunks (64 records, one per lane) per store. Keeping these agent-scope
// stores off the compute waves keeps their memory counter free of slow writes.
template <bool SUB, class Sh>
__device__ __attribute__((always_inline)) inline void out_helper(const DpArgs& a, Sh& sh, int ring_idx,
                                                                 int pl, uint64_t* rec, uint32_t tag) {
    const int lane = threadIdx.x & 63;
    const int64_t G = a.G;
    const float* ring = &sh.ring[ring_idx][0][0][0];
    const int q = lane >> 4, row = (lane & 15) >> 1, col = lane & 1;
    int prog_seen = 0;
    // panel pl publishes its band chunks, then +inf up to the last band
    // chunk of panel pl + 1
    const int64_t k0 = chunk_ranges<SUB>(pl, a.n, a.m, G).lo;
    const int64_t khi = chunk_ranges<SUB>(pl + 1, a.n, a.m, G).hi;
    if (lane == 0) lds_put(&sh.cons[ring_idx], int(k0));
    for (int64_t k = k0; k <= khi;) {
        if (prog_seen <= k) {
            int v;
            while ((v = lds_get(&sh.prog[ring_idx][0])) <= k) __builtin_amdgcn_s_sleep(1);
            prog_seen = v;
        }
        int avail = int(prog_seen - k) < 4 ? int(prog_seen - k) : 4;
        avail = khi + 1 - k < avail ? int(khi + 1 - k) : avail;
        compiler_order();
        float val = 0.0f;
        if (q < avail) val = ring[(int((k + q) % kRing) * 2 + col) * kChunk + row];
        compiler_order();
        if (lane == 0) lds_put(&sh.cons[ring_idx], int(k + avail));
        if (q < avail) {
            const uint64_t v = (uint64_t(tag) << 32) | uint64_t(__float_as_uint(val));
            __hip_atomic_store(rec + ((k + q) * kChunk + row) * 2 + col, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        k += avail;
    }
}

// The record column of boundary b (group b to b + 1) and the tag its records
// carry: the launch epoch and, when columns are reused, the lap's parity. A
// column is written again only after its previous boundary has been read in
// full, and band ranges only move down with the panel, so a slot holds this
// boundary's record, the previous lap's, or one of an earlier launch.
__device__ inline uint64_t* rec_column(const DpArgs& a, int b, int NW) {
    const int col = a.rec_slots > 0 ? b % a.rec_slots : b * NW + NW - 1;
    return a.rec + size_t(col) * size_t(a.G) * kChunk * 2;
}

__device__ inline uint32_t rec_tag(const DpArgs& a, int b, uint32_t epoch) {
    const uint32_t lap = a.rec_slots > 0 ? uint32_t(b / a.rec_slots) & 1u : 0u;
    return (epoch << 1) | lap;
}

// Panel group q (panels q*NW .. q*NW+NW-1) of one pair: NW compute waves, then
// the input helper and the output helper.
template <int NW, int SRC, bool SUB>
__device__ __attribute__((always_inline)) inline void run_group(const DpArgs& a, DpShared<NW>& sh, CostRing* cring,
                                                                int wave, int q, uint32_t epoch) {
    const int p0 = q * NW;
    if (wave < NW) {
        const int p = p0 + wave;
        if (p < a.P) compute_wave<SRC, SUB>(a, sh, cring, wave, p, p + 1 < a.P);
    } else if (is_fused(SRC) && wave >= NW + 2) {
        const int p = p0 + wave - (NW + 2);
        if constexpr (SRC == kSrcFusedB) {
            if (p < a.P) cost_producer_bf16(a, *cring, wave - (NW + 2), p, SUB);
        } else {
            if (p < a.P) cost_producer(a, *cring, wave - (NW + 2), p, SUB);
        }
    } else if (wave == NW) {
        if (p0 > 0) in_helper<SUB>(a, sh, p0 - 1, rec_column(a, q - 1, NW), rec_tag(a, q - 1, epoch));
        else inf_source(sh);
    } else {
        // the group's last panel feeds the next group when one exists
        if (p0 + NW < a.P) out_helper<SUB>(a, sh, NW, p0 + NW - 1, rec_column(a, q, NW), rec_tag(a, q, epoch));
    }
}

// Takes the next ticket and resets the group's LDS handoff counters.
template <int NW>
__device__ inline int next_ticket(DpShared<NW>& sh, CostRing* cring, DpWsHeader* hdr) {
    if (threadIdx.x == 0) {
        sh.super = int(atomicAdd(&hdr->ticket, 1u));
        for (int w = 0; w <= NW; ++w) { sh.prog[w][0] = 0; sh.prog[w][1] = 0; sh.cons[w] = 0; }
        if (cring)
            for (int w = 0; w < NW && w < kMaxNWFused; ++w) { cring->prog[w] = 0; cring->cons[w] = 0; }
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(sh.super);
}

constexpr int dp_waves(int nw, int src) { return is_fused(src) ? 2 * nw + 2 : nw + 2; }

template <int NW, int SRC, bool SUB>
__device__ __attribute__((always_inline)) inline void dp_body(const DpArgs& a, DpShared<NW>& sh, CostRing* cring) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes);
    const uint32_t epoch = __hip_atomic_load(&a.hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const int q = next_ticket<NW>(sh, cring, a.hdr);
        if (q >= a.S) break;
        run_group<NW, SRC, SUB>(a, sh, cring, wave, q, epoch);
        __syncthreads();
    }
}

template <int NW, int SRC, bool SUB>
__global__ __launch_bounds__(kLanes * dp_waves(NW, SRC)) void dp_kernel(DpArgs a) {
    __shared__ DpShared<NW> sh;
    if constexpr (is_fused(SRC)) {
        static_assert(NW <= kMaxNWFused, "fused workgroups hold at most kMaxNWFused compute waves");
        __shared__ CostRing cring;
        dp_body<NW, SRC, SUB>(a, sh, &cring);
    } else {
        dp_body<NW, SRC, SUB>(a, sh, nullptr);
    }
}

// Batched form: one persistent launch over the items of every pair. Items of
// one pair appear in increasing group order in the list, so a group again only
// waits on lower tickets.
struct DpBatchArgs {
    const BatchPair* pairs;
    const DpItem* items;
    int32_t nitems;
    const float* C;
    const float* X;    // fused cost: packed features and row norms
    const float* Y;
    const float* rxs;
    int64_t d;
    uint8_t* bp;
    float* totals;
    int32_t* status;
    DpWsHeader* hdr;
    uint64_t* rec;
};

template <int NW, int SRC, bool SUB>
__device__ __attribute__((always_inline)) inline void dp_batch_body(const DpBatchArgs& ba, DpShared<NW>& sh,
                                                                    CostRing* cring) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes);
    const uint32_t epoch = __hip_atomic_load(&ba.hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const int t = next_ticket<NW>(sh, cring, ba.hdr);
        if (t >= ba.nitems) break;
        const DpItem it = ba.items[t];
        const BatchPair q = ba.pairs[it.pair];
        DpArgs a;
        a.C = is_fused(SRC) ? nullptr : ba.C + q.c_off;
        a.X = is_fused(SRC) ? ba.X + q.x_off * ba.d : nullptr;
        a.Y = is_fused(SRC) ? ba.Y + q.y_off * ba.d : nullptr;
        a.rxs = SRC == kSrcFused ? ba.rxs + q.rx_off : nullptr;
        a.d = ba.d;
        a.bp = ba.bp + q.bp_off;
        // fragments of one plan share m: their score rows are stacked
        a.total = SUB ? ba.totals + int64_t(it.pair) * q.m : ba.totals + it.pair;
        a.status = ba.status + it.pair;
        a.hdr = ba.hdr;
        a.rec = ba.rec + q.rec_off;
        a.rec_slots = 0;
        a.n = q.n;
        a.m = q.m;
        a.G = q.G;
        a.P = q.P;
        a.S = int(ceil_div(q.P, NW));
        a.ckpt = nullptr;
        a.ck_chunks = 1;
        a.ck_count = 0;
        a.ck_stride = 0;
        run_group<NW, SRC, SUB>(a, sh, cring, wave, it.group, epoch);
        __syncthreads();
    }
}

template <int NW, int SRC, bool SUB>
__global__ __launch_bounds__(kLanes * dp_waves(NW, SRC)) void dp_batch_kernel(DpBatchArgs ba) {
    __shared__ DpShared<NW> sh;
    if constexpr (is_fused(SRC)) {
        static_assert(NW <= kMaxNWFused, "fused workgroups hold at most kMaxNWFused compute waves");
        __shared__ CostRing cring;
        dp_batch_body<NW, SRC, SUB>(ba, sh, &cring);
    } else {
        dp_batch_body<NW, SRC, SUB>(ba, sh, nullptr);
    }
}

// Row norms of pair b for the fused batched DP: blocks (b, y) for y <
// gridDim.y share the pair's rows, so one long pair is not left to one block.
__global__ void row_norms_batch_kernel(const BatchPair* __restrict__ pairs, const float* __restrict__ X, int64_t d,
                                       float* rxs) {
    const BatchPair q = pairs[blockIdx.x];
    if (!q.feasible) return;
    const int64_t len = rx_floats(q.n);
    for (int64_t i = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.y) * blockDim.x)
        rxs[q.rx_off + i] = row_inv_norm_f32_small(X + q.x_off * d, q.n, d, i);
}

// Segmental DTW with short fragments (at most kSweepRows rows, FP32 fused
// costs, d <= 16): one workgroup sweeps a whole fragment, each panel's chunks
// top to bottom. A fragment of 100 rows spans 13 chunks per panel, too few to
// pay for the handoffs and producer start-up of the staircase sweep. The
// workgroup's W waves take the panels in turn (wave w: panels w, w + W, ...),
// so that several waves share each SIMD and hide each other's latency; the
// two boundary columns of a panel pass to the next wave through LDS, chunk by
// chunk, with a count of finished chunks per wave. The fragment's row
// operands and norms stay in LDS for the whole sweep and each wave loads its
// next panel's column operands during the current one. The costs, the row
// step and the codes are those of the fused batched DP (the same slab code and
// row norms, the same dp_rows), so scores, codes and statuses are bit for bit
// the same. All of the fragment's chunks are swept: cells outside the
// subsequence band get exact values, which the band's argument makes
// irrelevant.
constexpr int kSweepRows = 256;

// LDS of one workgroup, sized at launch for R rows (the longest fragment's,
// rounded up to a whole 16-row slab), in this order:
//   cs   [W][2][kChunk * kLanes] each wave's slab costs (two chunks), panel layout
//   xs   [R][16]                 row operands, zero past d and n
//   rx   [R + 16]                row inverse norms, zero padded
//   bnd  [slots][2][R]           columns 64p-2 and 64p-1 of the panel to the left;
//                                slot w is written by wave w (one wave: two
//                                slots, used in turn)
//   done [W]                     chunks finished per wave
constexpr int sweep_slots(int W) { return W == 1 ? 2 : W; }
inline int sweep_rows(int64_t max_n) { return int((bp_groups(max_n) + 1) / 2) * 16; }
constexpr size_t sweep_lds_bytes(int W, int R) {
    return sizeof(float) * (size_t(W) * 2 * kChunk * kLanes + size_t(R) * 16 + R + 16 +
                            size_t(sweep_slots(W)) * 2 * R) + sizeof(int) * W;
}

struct FragSweepArgs {
    const BatchPair* pairs;
    const float* X;
    const float* Y;
    const float* rxs;
    int64_t d;
    uint8_t* bp;
    float* totals;   // [fragment][m] scores
    int32_t* status;
    int R;           // rows of the LDS arrays
};

// Slot reuse needs no flag of its own: wave w writes rows of chunk c of slot
// w for panel p only after the wave before it finished chunk c of panel p-1,
// which (around the ring of W waves) implies that wave w+1 finished chunk c of
// panel p-W+1, the last reader of the slot's previous contents. A wave reads
// only its own chunk's rows of a slot; the two rows above come in registers.
template <int W>
__global__ __launch_bounds__(kLanes * W, 3) void frag_sweep_kernel(FragSweepArgs a) {
    extern __shared__ f32x4 sweep_lds[];
    const int R = a.R;
    float* const cs = reinterpret_cast<float*>(sweep_lds);
    float* const xs = cs + W * 2 * kChunk * kLanes;
    float* const rxl = xs + R * 16;
    float* const bnd = rxl + R + 16;
    int* const done_l = reinterpret_cast<int*>(bnd + sweep_slots(W) * 2 * R);
    const int tid = threadIdx.x;
    const int lane = tid & (kLanes - 1);
    const int w = tid / kLanes;
    const int b = blockIdx.x;
    const BatchPair q = a.pairs[b];
    if (!q.feasible) return;  // scores and status set by the segment level's init
    const int n = int(q.n), G = int(q.G), P = q.P;
    const int64_t m = q.m, d = a.d;
    const float* X = a.X + q.x_off * d;
    const float* Y = a.Y + q.y_off * d;
    const float* rxs = a.rxs + q.rx_off;
    const float kInf = __builtin_inff();
    // rows of the fragment (and zero padding up to a whole slab)
    const int rows = ((G + 1) / 2) * 16;
    for (int e = tid; e < rows * 16; e += kLanes * W) {
        const int i = e >> 4, k = e & 15;
        xs[i * 16 + k] = (i < n && k < d) ? X[int64_t(i) * d + k] : 0.0f;
    }
    for (int i = tid; i < rows; i += kLanes * W) rxl[i] = i < n ? rxs[i] : 0.0f;
    // the slot that panel 0 reads: left of column 0 nothing is reachable
    constexpr int kFirst = W == 1 ? 0 : W - 1;
    for (int i = tid; i < G * kChunk; i += kLanes * W) {
        bnd[(kFirst * 2 + 0) * R + i] = kInf;
        bnd[(kFirst * 2 + 1) * R + i] = kInf;
    }
    if (tid < W) done_l[tid] = 0;
    const int g = lane >> 4;
    const int kq = lane >> 5, half = (lane >> 4) & 1, tcol = lane & 15;
    const int bcol = lane - (kLanes - 2);  // 0 / 1 on the two boundary lanes
    const int rlast = (n - 1) % kChunk;
    // the first panel's column operands
    float yn[4][4];
    auto load_panel = [&](int p, float (&yv)[4][4]) {
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            const int64_t col = int64_t(p) * kPanel + bb * 16 + (lane & 15);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t k = 4 * t + g;
                yv[bb][t] = (p < P && col < m && k < d) ? Y[col * d + k] : 0.0f;
            }
        }
    };
    load_panel(w, yn);
    __syncthreads();
    const int src = (w + W - 1) % W;  // the wave whose panels lie to the left of this wave's
    int cur = kFirst, done = 0, seen = 0;
    for (int p = w, kth = 0; p < P; p += W, ++kth) {
        // this panel's column operands and norms, as panel_operands_f32_small
        float bv[4][4], ry[4];
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            float sq = 0.0f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                bv[bb][t] = yn[bb][t];
                sq = __builtin_fmaf(bv[bb][t], bv[bb][t], sq);
            }
            ry[bb] = inv_from_sq(sum_groups(sq));
        }
        load_panel(p + W, yn);  // in flight during this panel
        const int put = W == 1 ? (cur ^ 1) : w;
        // chunks the source wave has finished once panel p-1's chunk c is done
        const int need0 = (w > 0 ? kth : kth - 1) * G + 1;
        float d1 = kInf, s1p = kInf, e0 = kInf, e1 = kInf, dlast = kInf;
        for (int k = 0; k < G; k += 2) {
            // the slab of chunks k and k + 1
            {
                float av[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) av[t] = xs[(8 * k + (lane & 15)) * 16 + 4 * t + g];
                const f32x4 rx4 = *reinterpret_cast<const f32x4*>(&rxl[8 * k + 4 * g]);
                f32x4 acc[4], v[4];
                slab_acc_f32_small(d, av, bv, acc);
                costs_from_acc_rx(acc, rx4, ry, v);
                float* dst = cs + (w * 2 + kq) * (kChunk * kLanes) + half * (kLanes * 4);
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) *reinterpret_cast<f32x4*>(dst + (bb * 16 + tcol) * 4) = v[bb];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int kk = k + u;
                if (kk >= G) break;
                float cb[kChunk], lv0[kChunk], lv1[kChunk];
                {
                    const f32x4* s4 = reinterpret_cast<const f32x4*>(cs + (w * 2 + u) * (kChunk * kLanes)) + lane;
                    const f32x4 c0 = s4[0], c1 = s4[kLanes];
                    cb[0] = c0[0]; cb[1] = c0[1]; cb[2] = c0[2]; cb[3] = c0[3];
                    cb[4] = c1[0]; cb[5] = c1[1]; cb[6] = c1[2]; cb[7] = c1[3];
                }
                if (W > 1 && p > 0) {
                    const int need = need0 + kk;
                    while (seen < need) {
                        seen = lds_get(&done_l[src]);
                        if (seen < need) __builtin_amdgcn_s_sleep(1);
                    }
                    compiler_order();
                }
                const int get = W == 1 ? cur : src;
#pragma unroll
                for (int r = 0; r < kChunk; ++r) {
                    lv0[r] = bnd[(get * 2 + 0) * R + kChunk * kk + r];
                    lv1[r] = bnd[(get * 2 + 1) * R + kChunk * kk + r];
                }
                // row 0 of the fragment: every cell a start, fma(2, C, -C) = C
                if (kk == 0) s1p = -cb[0];
                uint32_t lo, hi;
                float best_r[kChunk];
                dp_rows<true, false>(cb, lv0, lv1, e0, e1, d1, s1p, lo, hi, best_r);
                if (kk == 0) lo = (lo & ~0xffu) | 3u;
                e0 = lv0[kChunk - 1];
                e1 = lv1[kChunk - 1];
                uint64_t* cdst = reinterpret_cast<uint64_t*>(a.bp + q.bp_off) + (int64_t(p) * G + kk) * kLanes;
                cdst[lane] = uint64_t(lo) | (uint64_t(hi) << 32);
                if (bcol >= 0) {
#pragma unroll
                    for (int r = 0; r < kChunk; ++r) bnd[(put * 2 + bcol) * R + kChunk * kk + r] = best_r[r];
                }
                if constexpr (W > 1) {
                    compiler_order();
                    ++done;
                    if (lane == 0) lds_put(&done_l[w], done);
                }
                if (kk == G - 1) {
#pragma unroll
                    for (int r = 0; r < kChunk; ++r) dlast = (r == rlast) ? best_r[r] : dlast;
                }
            }
        }
        const int64_t col = int64_t(p) * kPanel + lane;
        if (col < m) a.totals[int64_t(b) * m + col] = dlast;
        if (col == m - 1) a.status[b] = dlast == kInf ? PARDTW_PAIR_INFEASIBLE : PARDTW_PAIR_OK;
        cur = put;
    }
}

// Row inverse norms for the fused producers (zeros past n, up to len).
__global__ void row_norms_kernel(const float* __restrict__ X, int64_t n, int64_t d, float* rxs, int64_t len) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < len; i += int64_t(gridDim.x) * blockDim.x)
        rxs[i] = row_inv_norm_f32_small(X, n, d, i);
}

__global__ void dp_prepare(DpWsHeader* hdr) {
    hdr->epoch = hdr->epoch + 1;
    hdr->ticket = 0;
}

// No path reaches (n-1, m-1) (or, for subsequence DTW, row n-1): the band is
// empty and nothing is swept; the `count` outputs are +inf.
__global__ void dp_infeasible(float* total, int64_t count, int32_t* status) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x)
        total[e] = __builtin_inff();
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = PARDTW_PAIR_INFEASIBLE;
}

int choose_nw(int P) {
    // Four panels per workgroup (one compute wave per SIMD) measured fastest
    // from 188 panels (12000 columns) up; tiny problems keep fewer.
    if (P >= 4) return 4;
    if (P >= 2) return 2;
    return 1;
}

template <int NW, int SRC>
void launch_src(const DpArgs& a, bool sub, int grid, hipStream_t stream) {
    if (sub) dp_kernel<NW, SRC, true><<<grid, kLanes * dp_waves(NW, SRC), 0, stream>>>(a);
    else dp_kernel<NW, SRC, false><<<grid, kLanes * dp_waves(NW, SRC), 0, stream>>>(a);
}

template <int NW>
void launch_nw(const DpArgs& a, int src, bool sub, int grid, hipStream_t stream) {
    if (src == kSrcPanel) launch_src<NW, kSrcPanel>(a, sub, grid, stream);
    else if (src == kSrcRow) launch_src<NW, kSrcRow>(a, sub, grid, stream);
    else if (src == kSrcPanelPk) dp_kernel<NW, kSrcPanelPk, false><<<grid, kLanes * dp_waves(NW, src), 0, stream>>>(a);
    else if constexpr (NW <= kMaxNWFused) {
        if (src == kSrcFused) launch_src<NW, kSrcFused>(a, sub, grid, stream);
        else if (src == kSrcFusedPk)
            dp_kernel<NW, kSrcFusedPk, false><<<grid, kLanes * dp_waves(NW, kSrcFusedPk), 0, stream>>>(a);
        else dp_kernel<NW, kSrcFusedCk, false><<<grid, kLanes * dp_waves(NW, kSrcFusedCk), 0, stream>>>(a);
    }
}

template <int NW, int SRC>
void launch_batch_src(const DpBatchArgs& a, bool sub, int grid, hipStream_t stream) {
    if (sub) dp_batch_kernel<NW, SRC, true><<<grid, kLanes * dp_waves(NW, SRC), 0, stream>>>(a);
    else dp_batch_kernel<NW, SRC, false><<<grid, kLanes * dp_waves(NW, SRC), 0, stream>>>(a);
}

template <int NW>
void launch_batch_nw(const DpBatchArgs& a, bool fused, bool bf16, bool sub, int grid, hipStream_t stream) {
    if (!fused) launch_batch_src<NW, kSrcPanel>(a, sub, grid, stream);
    else if constexpr (NW <= kMaxNWFusedB) {
        if (bf16) launch_batch_src<NW, kSrcFusedB>(a, sub, grid, stream);
        else launch_batch_src<NW, kSrcFused>(a, sub, grid, stream);
    } else if constexpr (NW <= kMaxNWFused) launch_batch_src<NW, kSrcFused>(a, sub, grid, stream);
}

}  // namespace

size_t dp_header_bytes() { return sizeof(DpWsHeader); }

// The DP reads only band groups, so the panel layouts are the same to it.
int src_of(pardtw_layout layout) { return layout == PARDTW_LAYOUT_ROW ? kSrcRow : kSrcPanel; }

// Batched pairs: one record column per panel.
size_t dp_record_bytes(int64_t n, int64_t m) {
    return size_t(num_panels(m)) * size_t(bp_groups(n)) * kChunk * 2 * sizeof(uint64_t);
}

// One pair: kRecSlots columns at most, whatever the panels per workgroup.
size_t dp_pair_record_bytes(int64_t n, int64_t m) {
    const int64_t cols = num_panels(m) < kRecSlots ? num_panels(m) : kRecSlots;
    return size_t(cols) * size_t(bp_groups(n)) * kChunk * 2 * sizeof(uint64_t);
}

size_t dp_workspace_bytes_impl(int64_t n, int64_t m) {
    return sizeof(DpWsHeader) + dp_pair_record_bytes(n, m) + size_t(rx_floats(n)) * sizeof(float);
}

pardtw_status dp_batch_launch(const BatchPair* pairs, const DpItem* items, int32_t nitems, int nw, int grid,
                              const float* Cbase, const float* X, const float* Y, int64_t d, const float* rxs,
                              bool bf16, uint8_t* bpbase, float* totals, int32_t* status, void* dp_ws, bool sub,
                              hipStream_t stream) {
    const bool fused = X != nullptr;
    if (fused && nw > (bf16 ? kMaxNWFusedB : kMaxNWFused)) return PARDTW_ERR_UNSUPPORTED;
    if (fused && bf16 && (d > 128 || d % 8 != 0)) return PARDTW_ERR_UNSUPPORTED;
    DpBatchArgs a;
    a.pairs = pairs;
    a.items = items;
    a.nitems = nitems;
    a.C = Cbase;
    a.X = X;
    a.Y = Y;
    a.rxs = rxs;
    a.d = d;
    a.bp = bpbase;
    a.totals = totals;
    a.status = status;
    a.hdr = reinterpret_cast<DpWsHeader*>(dp_ws);
    a.rec = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(dp_ws) + sizeof(DpWsHeader));
    dp_prepare<<<1, 1, 0, stream>>>(a.hdr);
    if (nitems <= 0) return launch_status();
    if (grid > nitems) grid = nitems;
    switch (nw) {
        case 1: launch_batch_nw<1>(a, fused, bf16, sub, grid, stream); break;
        case 2: launch_batch_nw<2>(a, fused, bf16, sub, grid, stream); break;
        case 4: launch_batch_nw<4>(a, fused, bf16, sub, grid, stream); break;
        case 8: launch_batch_nw<8>(a, fused, bf16, sub, grid, stream); break;
        default: return PARDTW_ERR_UNSUPPORTED;
    }
    return launch_status();
}

int64_t frag_sweep_max_rows() { return kSweepRows; }

pardtw_status frag_sweep_launch(const BatchPair* pairs, int32_t nfrag, int64_t max_n, int waves, const float* X,
                                const float* Y, int64_t d, const float* rxs, uint8_t* bpbase, float* totals,
                                int32_t* status, hipStream_t stream) {
    if (nfrag <= 0) return PARDTW_OK;
    if (max_n > kSweepRows || d > 16 || !X || !Y || !rxs) return PARDTW_ERR_UNSUPPORTED;
    FragSweepArgs a;
    a.pairs = pairs;
    a.X = X;
    a.Y = Y;
    a.rxs = rxs;
    a.d = d;
    a.bp = bpbase;
    a.totals = totals;
    a.status = status;
    a.R = sweep_rows(max_n);
    const size_t lds = sweep_lds_bytes(waves, a.R);
    switch (waves) {
        case 1: frag_sweep_kernel<1><<<unsigned(nfrag), kLanes, lds, stream>>>(a); break;
        case 2: frag_sweep_kernel<2><<<unsigned(nfrag), 2 * kLanes, lds, stream>>>(a); break;
        case 4: frag_sweep_kernel<4><<<unsigned(nfrag), 4 * kLanes, lds, stream>>>(a); break;
        default: return PARDTW_ERR_UNSUPPORTED;
    }
    return launch_status();
}

pardtw_status row_norms_batch_launch(const BatchPair* pairs, int32_t batch, int64_t max_n, const float* X,
                                     int64_t d, float* rxs, hipStream_t stream) {
    if (batch <= 0) return PARDTW_OK;
    const int64_t per = ceil_div(rx_floats(max_n > 0 ? max_n : 1), int64_t(256));
    const dim3 grid(unsigned(batch), unsigned(per < 64 ? per : 64));
    row_norms_batch_kernel<<<grid, 256, 0, stream>>>(pairs, X, d, rxs);
    return launch_status();
}

// src: the cost source (row-major or panel C, or fused from X, Y).
pardtw_status dp_launch(const float* C, const float* X, const float* Y, int64_t d, int src, int64_t n, int64_t m,
                        uint8_t* bp, float* total, int32_t* status, void* ws, int nw_override, bool sub,
                        hipStream_t stream, float* ckpt = nullptr, int ck_rows = 0) {
    DpArgs a;
    a.C = C;
    a.X = X;
    a.Y = Y;
    a.d = d;
    a.bp = bp;
    a.total = total;
    a.status = status;
    a.hdr = reinterpret_cast<DpWsHeader*>(ws);
    a.rec = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(ws) + sizeof(DpWsHeader));
    // the records are a multiple of 128 bytes, so the row-norm area is 16-byte aligned
    a.rxs = reinterpret_cast<float*>(reinterpret_cast<char*>(a.rec) + dp_pair_record_bytes(n, m));
    a.n = n;
    a.m = m;
    a.G = bp_groups(n);
    a.P = int(num_panels(m));
    const int nw = nw_override > 0 ? nw_override : choose_nw(a.P);
    a.S = int(ceil_div(a.P, nw));
    int dev = 0, cus = 0;
    PARDTW_HIP_TRY(hipGetDevice(&dev));
    PARDTW_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // about four compute waves per CU (one per SIMD)
    const int per_cu = nw >= 4 ? 1 : 4 / nw;
    int grid = a.S < cus * per_cu ? a.S : cus * per_cu;
    // the record columns must outnumber the groups in flight
    grid = grid < kRecSlots - 1 ? grid : kRecSlots - 1;
    a.rec_slots = a.S < kRecSlots ? a.S : kRecSlots;
    if (is_fused(src) && nw > kMaxNWFused) return PARDTW_ERR_UNSUPPORTED;
    if (src == kSrcFusedCk && (sub || ck_rows < 16 || ck_rows > kCkMaxRows || ck_rows % 16))
        return PARDTW_ERR_INVALID_ARG;
    a.ckpt = ckpt;
    a.ck_chunks = ck_rows > 0 ? ck_rows / kChunk : 1;
    a.ck_count = src == kSrcFusedCk ? int(ckpt_count(n, ck_rows)) : 0;
    if (a.ck_count > 0 && !ckpt) return PARDTW_ERR_INVALID_ARG;
    a.ck_stride = int64_t(a.P) * kPanel;
    if (sub ? !subseq_feasible(n, m) : !pair_feasible(n, m)) {
        const int64_t count = sub ? m : 1;
        const unsigned blocks = unsigned(count < 256 * 1024 ? ceil_div(count, 256) : 1024);
        dp_infeasible<<<blocks, 256, 0, stream>>>(total, count, status);
        return launch_status();
    }
    dp_prepare<<<1, 1, 0, stream>>>(a.hdr);
    if (is_fused(src)) {
        const int64_t len = rx_floats(n);
        const unsigned blocks = unsigned(len < 256 * 2048 ? ceil_div(len, 256) : 2048);
        row_norms_kernel<<<blocks, 256, 0, stream>>>(X, n, d, const_cast<float*>(a.rxs), len);
    }
    switch (nw) {
        case 1: launch_nw<1>(a, src, sub, grid, stream); break;
        case 2: launch_nw<2>(a, src, sub, grid, stream); break;
        case 4: launch_nw<4>(a, src, sub, grid, stream); break;
        case 8: launch_nw<8>(a, src, sub, grid, stream); break;
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
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL && layout != PARDTW_LAYOUT_PANEL_BAND)
        return PARDTW_ERR_UNSUPPORTED;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(C, nullptr, nullptr, 0, pardtw::src_of(layout), n, m, bp, total, pair_status,
                             workspace, 0, false, stream);
}

extern "C" pardtw_status pardtw_dp_ex(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                                      float* total, int32_t* pair_status, void* workspace, size_t workspace_bytes,
                                      int32_t panels_per_workgroup, hipStream_t stream) {
    if (!C || !bp || !total || !pair_status || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL && layout != PARDTW_LAYOUT_PANEL_BAND)
        return PARDTW_ERR_UNSUPPORTED;
    if (panels_per_workgroup != 0 && panels_per_workgroup != 1 && panels_per_workgroup != 2 &&
        panels_per_workgroup != 4 && panels_per_workgroup != 8)
        return PARDTW_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(C, nullptr, nullptr, 0, pardtw::src_of(layout), n, m, bp, total, pair_status,
                             workspace, panels_per_workgroup, false, stream);
}

extern "C" pardtw_status pardtw_subseq_dp(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                                          float* scores, int32_t* pair_status, void* workspace,
                                          size_t workspace_bytes, hipStream_t stream) {
    if (!C || !bp || !scores || !pair_status || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL && layout != PARDTW_LAYOUT_PANEL_SUBSEQ_BAND)
        return PARDTW_ERR_UNSUPPORTED;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(C, nullptr, nullptr, 0, pardtw::src_of(layout), n, m, bp, scores, pair_status,
                             workspace, 0, true, stream);
}

namespace {

// Device address of `scratch` per device, taken on the first call on that
// device with the device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];

pardtw_status scratch_address(void** out) {
    int dev = 0;
    PARDTW_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return PARDTW_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PARDTW_ERR_HIP;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return PARDTW_OK;
}

pardtw_status check_fused(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, uint8_t* bp, float* out,
                          int32_t* st, void* ws, size_t ws_bytes, int32_t nw) {
    if (!X || !Y || !bp || !out || !st || !pardtw::valid_sizes(n, m) || d <= 0) return PARDTW_ERR_INVALID_ARG;
    if (d > 16) return PARDTW_ERR_UNSUPPORTED;
    if (nw != 0 && nw != 1 && nw != 2 && nw != 4) return PARDTW_ERR_INVALID_ARG;
    if (!ws || ws_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return PARDTW_OK;
}

}  // namespace

extern "C" pardtw_status pardtw_dp_fused(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                         uint8_t* bp, float* total, int32_t* pair_status, void* workspace,
                                         size_t workspace_bytes, int32_t panels_per_workgroup, hipStream_t stream) {
    const pardtw_status st = check_fused(X, Y, n, m, d, bp, total, pair_status, workspace, workspace_bytes,
                                         panels_per_workgroup);
    if (st != PARDTW_OK) return st;
    return pardtw::dp_launch(nullptr, X, Y, d, pardtw::kSrcFused, n, m, bp, total, pair_status, workspace,
                             panels_per_workgroup, false, stream);
}

extern "C" pardtw_status pardtw_dp_fused_ckpt(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                              int32_t rows_per_block, float* ckpt, size_t ckpt_bytes, float* total,
                                              int32_t* pair_status, void* workspace, size_t workspace_bytes,
                                              hipStream_t stream) {
    if (!X || !Y || !total || !pair_status || !pardtw::valid_sizes(n, m) || d <= 0) return PARDTW_ERR_INVALID_ARG;
    if (d > 16) return PARDTW_ERR_UNSUPPORTED;
    if (rows_per_block < 16 || rows_per_block > pardtw::kCkMaxRows || rows_per_block % 16)
        return PARDTW_ERR_INVALID_ARG;
    const int64_t floats = pardtw::ckpt_floats(n, m, rows_per_block);
    if (floats > 0 && (!ckpt || ckpt_bytes < size_t(floats) * sizeof(float))) return PARDTW_ERR_WORKSPACE;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(nullptr, X, Y, d, pardtw::kSrcFusedCk, n, m, nullptr, total, pair_status, workspace, 0,
                             false, stream, ckpt, rows_per_block);
}

extern "C" pardtw_status pardtw_subseq_dp_fused(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                                uint8_t* bp, float* scores, int32_t* pair_status, void* workspace,
                                                size_t workspace_bytes, hipStream_t stream) {
    const pardtw_status st = check_fused(X, Y, n, m, d, bp, scores, pair_status, workspace, workspace_bytes, 0);
    if (st != PARDTW_OK) return st;
    return pardtw::dp_launch(nullptr, X, Y, d, pardtw::kSrcFused, n, m, bp, scores, pair_status, workspace, 0, true,
                             stream);
}

extern "C" pardtw_status pardtw_dp_noalloc(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint8_t* bp,
                                           float* total, int32_t* pair_status, hipStream_t stream) {
    if (!C || !bp || !total || !pair_status || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (layout != PARDTW_LAYOUT_ROW && layout != PARDTW_LAYOUT_PANEL && layout != PARDTW_LAYOUT_PANEL_BAND)
        return PARDTW_ERR_UNSUPPORTED;
    if (pardtw::dp_workspace_bytes_impl(n, m) > size_t(PARDTW_NOALLOC_SCRATCH_BYTES)) return PARDTW_ERR_WORKSPACE;
    void* ws = nullptr;
    if (const pardtw_status st = scratch_address(&ws); st != PARDTW_OK) return st;
    return pardtw::dp_launch(C, nullptr, nullptr, 0, pardtw::src_of(layout), n, m, bp, total, pair_status, ws, 0,
                             false, stream);
}

extern "C" size_t pardtw_bp2_bytes(int64_t n, int64_t m) {
    if (!pardtw::valid_sizes(n, m)) return 0;
    return size_t(pardtw::num_panels(m)) * size_t(pardtw::bp_groups(n)) * pardtw::kLanes * sizeof(uint16_t);
}

extern "C" pardtw_status pardtw_dp_packed(const float* C, pardtw_layout layout, int64_t n, int64_t m, uint16_t* bp2,
                                          float* total, int32_t* pair_status, void* workspace,
                                          size_t workspace_bytes, hipStream_t stream) {
    if (!C || !bp2 || !total || !pair_status || !pardtw::valid_sizes(n, m)) return PARDTW_ERR_INVALID_ARG;
    if (layout != PARDTW_LAYOUT_PANEL && layout != PARDTW_LAYOUT_PANEL_BAND) return PARDTW_ERR_UNSUPPORTED;
    if (!workspace || workspace_bytes < pardtw::dp_workspace_bytes_impl(n, m)) return PARDTW_ERR_WORKSPACE;
    return pardtw::dp_launch(C, nullptr, nullptr, 0, pardtw::kSrcPanelPk, n, m, reinterpret_cast<uint8_t*>(bp2),
                             total, pair_status, workspace, 0, false, stream);
}

extern "C" pardtw_status pardtw_dp_fused_packed(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                                                uint16_t* bp2, float* total, int32_t* pair_status, void* workspace,
                                                size_t workspace_bytes, hipStream_t stream) {
    const pardtw_status st = check_fused(X, Y, n, m, d, reinterpret_cast<uint8_t*>(bp2), total, pair_status,
                                         workspace, workspace_bytes, 0);
    if (st != PARDTW_OK) return st;
    return pardtw::dp_launch(nullptr, X, Y, d, pardtw::kSrcFusedPk, n, m, reinterpret_cast<uint8_t*>(bp2), total,
                             pair_status, workspace, 0, false, stream);
}
