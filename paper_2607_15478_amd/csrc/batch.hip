// a5: batched form. A plan fixes the pair lengths of a batch, lays out one
// workspace for all of them, and holds in device memory what every kernel of
// the batch needs (pair descriptors, the cost tiles' pair table and the DP's
// work lists for each candidate schedule), so that pardtw_align_batch issues
// only kernel launches: no allocation, copy or host synchronisation, and it
// can be captured in a hipGraph.
//
// The DP of all pairs runs as one persistent launch drawing (pair, panel
// group) items from one ticket. A schedule fixes the panels per workgroup
// (1, 2, 4 or 8), the order of the items (breadth: group 0 of every pair, then
// group 1, ...; depth: every group of the largest pair, then the next) and the
// number of resident workgroups; pardtw_plan_autotune times each schedule on
// the caller's data and keeps the fastest.
//
// A Segmental DTW plan (Sec. II-C) reuses all of it: its pairs are the
// fragments of sequence A, each against the whole of sequence B, swept by the
// subsequence DP, followed by the segment-level program, the fragments'
// backtraces and their concatenation.
#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "batch.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Schedule {
    int nw;          // panels per workgroup; 0: one workgroup per fragment (frag_sweep_launch)
    int order;       // 0 breadth, 1 depth
    int grid_mul;    // resident workgroups per CU, relative to the NW default; nw 0: waves per fragment
    int32_t nitems;
    int64_t items_at;  // first item in the plan's item array
};

__global__ void batch_init_kernel(const pardtw::BatchPair* __restrict__ pairs, int32_t batch, float* totals,
                                  int32_t* status, int32_t* path_len) {
    const int b = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= batch || pairs[b].feasible) return;
    totals[b] = __builtin_inff();
    status[b] = PARDTW_PAIR_INFEASIBLE;
    path_len[b] = 0;
}

}  // namespace

struct pardtw_plan {
    int mode = 0;       // 0 independent pairs, 1 Segmental DTW fragments
    bool fused = false; // costs computed inside the DP: no cost region, a row-norm region instead
    int variant = 1;    // Segmental DTW: PARDTW_NSDTW or PARDTW_WSDTW
    int64_t la = 0, lb = 0, hop = 1;
    size_t off_s = 0, off_fstat = 0, off_slots = 0, off_flen = 0, off_seg = 0, off_rx = 0;
    int32_t batch = 0;
    int64_t d = 0;
    pardtw_prec prec = PARDTW_PREC_F32;
    int device = 0;
    int cus = 1;
    std::vector<pardtw::BatchPair> pairs;
    pardtw::BatchPair* pairs_dev = nullptr;
    int32_t* tile_pair_dev = nullptr;
    int64_t tiles = 0;
    pardtw::DpItem* items_dev = nullptr;
    std::vector<Schedule> scheds;
    int chosen = 0;
    size_t off_c = 0, off_bp = 0, off_dp = 0, ws_bytes = 0;
    int64_t path_capacity = 0, max_cap = 0, max_n = 0, x_rows = 0, y_rows = 0;
    // split backtraces of the long pairs: their segments and the workspace
    // region of their segment records and cells
    std::vector<pardtw::SegPair> segpairs;
    std::vector<int32_t> seg_map;
    pardtw::SegPair* segpairs_dev = nullptr;
    int32_t* seg_map_dev = nullptr;
    size_t off_split_rec = 0, off_split_cells = 0;

    ~pardtw_plan() {
        if (pairs_dev) (void)hipFree(pairs_dev);
        if (tile_pair_dev) (void)hipFree(tile_pair_dev);
        if (items_dev) (void)hipFree(items_dev);
        if (segpairs_dev) (void)hipFree(segpairs_dev);
        if (seg_map_dev) (void)hipFree(seg_map_dev);
    }
};

namespace {

int grid_for(const pardtw_plan& pl, const Schedule& s) {
    if (s.nw == 0) return int(pl.batch);
    const int per_cu = s.nw >= 4 ? 1 : 4 / s.nw;
    return pl.cus * per_cu * s.grid_mul;
}

// Work list of one schedule: items of each pair in increasing group order.
std::vector<pardtw::DpItem> make_items(const pardtw_plan& pl, int nw, int order) {
    std::vector<int> rank;
    for (int b = 0; b < pl.batch; ++b)
        if (pl.pairs[b].feasible) rank.push_back(b);
    std::stable_sort(rank.begin(), rank.end(), [&](int x, int y) {
        return pl.pairs[x].n * pl.pairs[x].m > pl.pairs[y].n * pl.pairs[y].m;
    });
    std::vector<pardtw::DpItem> items;
    if (order == 1) {
        for (int b : rank) {
            const int S = int(pardtw::ceil_div(pl.pairs[b].P, nw));
            for (int q = 0; q < S; ++q) items.push_back({b, q});
        }
    } else {
        int smax = 0;
        for (int b : rank) smax = std::max(smax, int(pardtw::ceil_div(pl.pairs[b].P, nw)));
        for (int q = 0; q < smax; ++q)
            for (int b : rank)
                if (q < pardtw::ceil_div(pl.pairs[b].P, nw)) items.push_back({b, q});
    }
    return items;
}

// A Segmental DTW plan's DP writes the fragments' scores and statuses into
// its workspace; `totals` / `status` serve plans of pairs. X, Y are the packed
// features, read by the fused form.
pardtw_status run_dp(const pardtw_plan& pl, const Schedule& s, char* ws, const float* X, const float* Y,
                     float* totals, int32_t* status, hipStream_t stream) {
    const bool sub = pl.mode == 1;
    if (sub) {
        totals = reinterpret_cast<float*>(ws + pl.off_s);
        status = reinterpret_cast<int32_t*>(ws + pl.off_fstat);
    }
    if (s.nw == 0)
        return pardtw::frag_sweep_launch(pl.pairs_dev, int32_t(pl.batch), pl.max_n, s.grid_mul, X, Y, pl.d,
                                         reinterpret_cast<const float*>(ws + pl.off_rx),
                                         reinterpret_cast<uint8_t*>(ws + pl.off_bp), totals, status, stream);
    return pardtw::dp_batch_launch(pl.pairs_dev, pl.items_dev + s.items_at, s.nitems, s.nw, grid_for(pl, s),
                                   reinterpret_cast<const float*>(ws + pl.off_c), pl.fused ? X : nullptr, Y, pl.d,
                                   reinterpret_cast<const float*>(ws + pl.off_rx), pl.prec == PARDTW_PREC_BF16,
                                   reinterpret_cast<uint8_t*>(ws + pl.off_bp), totals, status, ws + pl.off_dp, sub,
                                   stream);
}

// What precedes the DP: the cost GEMM, or for the FP32 fused form the row
// norms (the BF16 fused form takes them from its row operands).
pardtw_status run_front(const pardtw_plan& pl, const float* X, const float* Y, char* ws, hipStream_t stream) {
    if (pl.fused && pl.prec == PARDTW_PREC_BF16) return PARDTW_OK;
    if (pl.fused)
        return pardtw::row_norms_batch_launch(pl.pairs_dev, pl.batch, pl.max_n, X, pl.d,
                                              reinterpret_cast<float*>(ws + pl.off_rx), stream);
    return pardtw::cost_batch_launch(pl.pairs_dev, pl.tile_pair_dev, pl.tiles, X, Y, pl.d, pl.prec,
                                     reinterpret_cast<float*>(ws + pl.off_c), stream);
}

bool aligned(const void* p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; }

pardtw_status check_call(const pardtw_plan* plan, const float* X, const float* Y, void* ws, size_t ws_bytes,
                         float* totals, int32_t* paths, int32_t* path_len, int32_t* status) {
    if (!plan || !X || !Y || !ws || !totals || !paths || !path_len || !status) return PARDTW_ERR_INVALID_ARG;
    if (plan->mode != 0) return PARDTW_ERR_INVALID_ARG;
    if (!aligned(ws, kAlign) || !aligned(paths, 8)) return PARDTW_ERR_INVALID_ARG;
    if (ws_bytes < plan->ws_bytes) return PARDTW_ERR_WORKSPACE;
    return PARDTW_OK;
}

// Lays out one pair (or fragment) b: descriptor offsets into the cost (or,
// fused, row-norm), code and record regions, counted in the running totals.
void place_pair(pardtw::BatchPair& q, int64_t n, int64_t m, bool feasible, int band, bool fused, size_t& c_floats,
                size_t& bp_bytes, size_t& rec_bytes, size_t& rx_total, int64_t& tiles) {
    q.n = n;
    q.m = m;
    q.G = pardtw::bp_groups(n);
    q.P = int32_t(pardtw::num_panels(m));
    q.feasible = feasible ? 1 : 0;
    q.band = band;
    q.split = 0;
    q.c_off = int64_t(c_floats);
    q.bp_off = int64_t(bp_bytes);
    q.rec_off = int64_t(rec_bytes / sizeof(uint64_t));
    q.tile0 = tiles;
    q.rx_off = int64_t(rx_total);
    if (feasible) {
        const size_t cells = size_t(q.P) * size_t(q.G) * pardtw::kPanel * pardtw::kBpRows;
        bp_bytes += cells;  // multiples of 512: keeps every pair 256-byte aligned
        rec_bytes += pardtw::dp_record_bytes(n, m);
        if (fused) {
            rx_total += size_t(pardtw::ceil_div(pardtw::rx_floats(n), 64) * 64);  // 256-byte steps
        } else {
            c_floats += cells;
            tiles += pardtw::cost_blocks(n, m);
        }
    }
}

// The device tables of a laid-out plan: cost block -> pair table, the DP work
// lists of every candidate schedule, the pair descriptors.
pardtw_status finish_plan(pardtw_plan* pl, pardtw_plan** plan_out) {
    const int32_t batch = pl->batch;
    const int64_t tiles = pl->tiles;
    // cost block -> pair table of the batched cost kernel (none for the fused
    // form, which runs no cost kernel and counted no blocks)
    std::vector<int32_t> tile_pair(size_t(std::max<int64_t>(tiles, 1)));
    for (int b = 0; b < batch && !pl->fused; ++b) {
        const pardtw::BatchPair& q = pl->pairs[b];
        if (!q.feasible) continue;
        const int64_t t = pardtw::cost_blocks(q.n, q.m);
        std::fill(tile_pair.begin() + q.tile0, tile_pair.begin() + q.tile0 + t, b);
    }

    // candidate schedules and their work lists (fused workgroups hold at most
    // four compute waves). Segmental DTW fragments differ by one row at most,
    // so depth order would run them nearly one after another (hundreds of
    // times slower at 1000 fragments) and with one fragment it equals
    // breadth order: those plans try breadth order only.
    std::vector<pardtw::DpItem> all_items;
    const int nws[4] = {1, 2, 4, 8};
    const int orders = pl->mode == 1 ? 1 : 2;
    for (int nw : nws) {
        if (pl->fused && nw > (pl->prec == PARDTW_PREC_BF16 ? 2 : 4)) continue;
        for (int order = 0; order < orders; ++order) {
            const std::vector<pardtw::DpItem> it = make_items(*pl, nw, order);
            const int64_t at = int64_t(all_items.size());
            all_items.insert(all_items.end(), it.begin(), it.end());
            for (int gm = 1; gm <= 2; ++gm) pl->scheds.push_back({nw, order, gm, int32_t(it.size()), at});
        }
    }
    // default: four panels per workgroup (two for BF16 fused), breadth order,
    // one workgroup per CU
    const int nw_default = pl->fused && pl->prec == PARDTW_PREC_BF16 ? 2 : 4;
    pl->chosen = 0;
    for (size_t s = 0; s < pl->scheds.size(); ++s)
        if (pl->scheds[s].nw == nw_default && pl->scheds[s].order == 0 && pl->scheds[s].grid_mul == 1)
            pl->chosen = int(s);
    // Segmental DTW with short fragments and fused FP32 costs: also one
    // workgroup per fragment sweeping all of its panels, with 1, 2 or 4 waves
    // taking them in turn (no handoffs between workgroups)
    if (pl->mode == 1 && pl->fused && pl->prec == PARDTW_PREC_F32 && pl->d <= 16 &&
        pl->max_n <= pardtw::frag_sweep_max_rows())
        for (int waves : {1, 2, 4}) pl->scheds.push_back({0, 0, waves, 0, 0});
    if (all_items.empty()) all_items.push_back({0, 0});

    bool ok = hipMalloc(&pl->pairs_dev, sizeof(pardtw::BatchPair) * batch) == hipSuccess &&
              hipMalloc(&pl->tile_pair_dev, sizeof(int32_t) * tile_pair.size()) == hipSuccess &&
              hipMalloc(&pl->items_dev, sizeof(pardtw::DpItem) * all_items.size()) == hipSuccess;
    ok = ok && hipMemcpy(pl->pairs_dev, pl->pairs.data(), sizeof(pardtw::BatchPair) * batch,
                         hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->tile_pair_dev, tile_pair.data(), sizeof(int32_t) * tile_pair.size(),
                         hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(pl->items_dev, all_items.data(), sizeof(pardtw::DpItem) * all_items.size(),
                         hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !pl->segpairs.empty()) {
        ok = hipMalloc(&pl->segpairs_dev, sizeof(pardtw::SegPair) * pl->segpairs.size()) == hipSuccess &&
             hipMalloc(&pl->seg_map_dev, sizeof(int32_t) * pl->seg_map.size()) == hipSuccess &&
             hipMemcpy(pl->segpairs_dev, pl->segpairs.data(), sizeof(pardtw::SegPair) * pl->segpairs.size(),
                       hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(pl->seg_map_dev, pl->seg_map.data(), sizeof(int32_t) * pl->seg_map.size(),
                       hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        delete pl;
        return PARDTW_ERR_HIP;
    }
    *plan_out = pl;
    return PARDTW_OK;
}

}  // namespace

namespace {

// The fused form computes FP32 costs from features with at most 16 entries,
// or BF16-operand costs from features with at most 128 entries, a multiple of 8.
pardtw_status check_flags(int32_t flags, int64_t d, pardtw_prec prec) {
    if (flags & ~int32_t(PARDTW_PLAN_FUSED_COST)) return PARDTW_ERR_INVALID_ARG;
    if (flags & PARDTW_PLAN_FUSED_COST) {
        const bool f32_ok = prec == PARDTW_PREC_F32 && d <= 16;
        const bool bf16_ok = prec == PARDTW_PREC_BF16 && d <= 128 && d % 8 == 0;
        if (!f32_ok && !bf16_ok) return PARDTW_ERR_UNSUPPORTED;
    }
    return PARDTW_OK;
}

}  // namespace

extern "C" pardtw_status pardtw_plan_create(int32_t batch, const int64_t* n_host, const int64_t* m_host, int64_t d,
                                            pardtw_prec prec, pardtw_plan** plan_out) {
    return pardtw_plan_create_ex(batch, n_host, m_host, d, prec, 0, plan_out);
}

extern "C" pardtw_status pardtw_plan_create_ex(int32_t batch, const int64_t* n_host, const int64_t* m_host,
                                               int64_t d, pardtw_prec prec, int32_t flags, pardtw_plan** plan_out) {
    if (!plan_out) return PARDTW_ERR_INVALID_ARG;
    *plan_out = nullptr;
    if (batch <= 0 || !n_host || !m_host || d <= 0 || d > (int64_t(1) << 20)) return PARDTW_ERR_INVALID_ARG;
    if (prec != PARDTW_PREC_F32 && prec != PARDTW_PREC_BF16) return PARDTW_ERR_UNSUPPORTED;
    if (const pardtw_status fs = check_flags(flags, d, prec); fs != PARDTW_OK) return fs;
    for (int b = 0; b < batch; ++b)
        if (!pardtw::valid_sizes(n_host[b], m_host[b])) return PARDTW_ERR_INVALID_ARG;

    pardtw_plan* pl = new (std::nothrow) pardtw_plan;
    if (!pl) return PARDTW_ERR_HIP;
    pl->batch = batch;
    pl->d = d;
    pl->prec = prec;
    pl->fused = (flags & PARDTW_PLAN_FUSED_COST) != 0;
    if (hipGetDevice(&pl->device) != hipSuccess ||
        hipDeviceGetAttribute(&pl->cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess) {
        delete pl;
        return PARDTW_ERR_HIP;
    }

    // descriptors and the workspace layout: cost panels (or row norms) | codes |
    // DP header + records
    pl->pairs.resize(batch);
    size_t c_floats = 0, bp_bytes = 0, rec_bytes = 0, rx_total = 0;
    int64_t xr = 0, yr = 0, po = 0, tiles = 0;
    for (int b = 0; b < batch; ++b) {
        pardtw::BatchPair& q = pl->pairs[b];
        const int64_t n = n_host[b], m = m_host[b];
        q.x_off = xr;
        q.y_off = yr;
        q.path_off = po;
        place_pair(q, n, m, pardtw::pair_feasible(n, m), 1, pl->fused, c_floats, bp_bytes, rec_bytes, rx_total, tiles);
        const int64_t cap = std::min(n, m);
        xr += n;
        yr += m;
        po += cap;
        pl->max_cap = std::max(pl->max_cap, cap);
        pl->max_n = std::max(pl->max_n, n);
    }
    pl->x_rows = xr;
    pl->y_rows = yr;
    pl->path_capacity = po;
    pl->tiles = tiles;
    pl->off_c = 0;
    pl->off_rx = 0;  // the fused form's row norms take the cost region's place
    pl->off_bp = align_up((pl->fused ? rx_total : c_floats) * sizeof(float));
    pl->off_dp = pl->off_bp + align_up(bp_bytes);
    // pairs of more than two segments get the split walk (pardtw_backtrace_parallel's)
    int64_t nrec = 0, ncells = 0;
    for (int b = 0; b < batch; ++b) {
        pardtw::BatchPair& q = pl->pairs[b];
        int R, S;
        pardtw::split_shape(q.n, R, S);
        if (!q.feasible || S <= 2) continue;
        q.split = 1;
        const int32_t idx = int32_t(pl->segpairs.size());
        pl->segpairs.push_back({b, R, S, int32_t(pl->seg_map.size()), nrec, ncells});
        pl->seg_map.insert(pl->seg_map.end(), size_t(S), idx);
        nrec += 2 * int64_t(S);
        ncells += int64_t(S) * R * 2;
    }
    pl->off_split_rec = pl->off_dp + align_up(pardtw::dp_header_bytes() + rec_bytes);
    pl->off_split_cells = pl->off_split_rec + align_up(size_t(nrec) * pardtw::split_record_bytes());
    pl->ws_bytes = pl->off_split_cells + align_up(size_t(ncells) * sizeof(int32_t));
    return finish_plan(pl, plan_out);
}


extern "C" size_t pardtw_plan_workspace_bytes(const pardtw_plan* plan) { return plan ? plan->ws_bytes : 0; }

extern "C" int64_t pardtw_plan_path_capacity(const pardtw_plan* plan) { return plan ? plan->path_capacity : 0; }

extern "C" void pardtw_plan_destroy(pardtw_plan* plan) { delete plan; }

extern "C" int32_t pardtw_plan_num_schedules(const pardtw_plan* plan) {
    return plan ? int32_t(plan->scheds.size()) : 0;
}

extern "C" pardtw_status pardtw_plan_schedule(const pardtw_plan* plan, int32_t index, int32_t* panels_per_workgroup,
                                              int32_t* order, int32_t* workgroups) {
    if (!plan || index < -1 || index >= int32_t(plan->scheds.size())) return PARDTW_ERR_INVALID_ARG;
    const Schedule& s = plan->scheds[index < 0 ? plan->chosen : index];
    if (panels_per_workgroup) *panels_per_workgroup = s.nw;
    if (order) *order = s.nw == 0 ? s.grid_mul : s.order;
    if (workgroups) *workgroups = s.nw == 0 ? grid_for(*plan, s) : std::min(grid_for(*plan, s), std::max(s.nitems, 1));
    return PARDTW_OK;
}

extern "C" int32_t pardtw_plan_selected(const pardtw_plan* plan) { return plan ? plan->chosen : -1; }

extern "C" pardtw_status pardtw_plan_select(pardtw_plan* plan, int32_t index) {
    if (!plan || index < 0 || index >= int32_t(plan->scheds.size())) return PARDTW_ERR_INVALID_ARG;
    plan->chosen = index;
    return PARDTW_OK;
}

extern "C" pardtw_status pardtw_align_batch(const pardtw_plan* plan, const float* X_packed, const float* Y_packed,
                                            void* workspace, size_t workspace_bytes, float* totals,
                                            int32_t* paths_packed, int32_t* path_len, int32_t* pair_status,
                                            hipStream_t stream) {
    pardtw_status st = check_call(plan, X_packed, Y_packed, workspace, workspace_bytes, totals, paths_packed,
                                  path_len, pair_status);
    if (st != PARDTW_OK) return st;
    char* ws = static_cast<char*>(workspace);
    batch_init_kernel<<<unsigned(pardtw::ceil_div(plan->batch, 256)), 256, 0, stream>>>(
        plan->pairs_dev, plan->batch, totals, pair_status, path_len);
    if ((st = pardtw::launch_status()) != PARDTW_OK) return st;
    st = run_front(*plan, X_packed, Y_packed, ws, stream);
    if (st != PARDTW_OK) return st;
    st = run_dp(*plan, plan->scheds[plan->chosen], ws, X_packed, Y_packed, totals, pair_status, stream);
    if (st != PARDTW_OK) return st;
    const uint8_t* bp = reinterpret_cast<const uint8_t*>(ws + plan->off_bp);
    st = pardtw::backtrace_batch_launch(plan->pairs_dev, plan->batch, bp, pair_status, paths_packed, path_len,
                                        stream);
    if (st != PARDTW_OK) return st;
    return pardtw::split_backtrace_batch_launch(plan->pairs_dev, plan->segpairs_dev, int32_t(plan->segpairs.size()),
                                                plan->seg_map_dev, int32_t(plan->seg_map.size()), bp, pair_status,
                                                nullptr, ws + plan->off_split_rec,
                                                reinterpret_cast<int32_t*>(ws + plan->off_split_cells),
                                                paths_packed, path_len, stream);
}

extern "C" pardtw_status pardtw_plan_autotune(pardtw_plan* plan, const float* X_packed, const float* Y_packed,
                                              void* workspace, size_t workspace_bytes, float* totals,
                                              int32_t* paths_packed, int32_t* path_len, int32_t* pair_status,
                                              int32_t reps, float* best_ms, hipStream_t stream) {
    pardtw_status st = check_call(plan, X_packed, Y_packed, workspace, workspace_bytes, totals, paths_packed,
                                  path_len, pair_status);
    if (st != PARDTW_OK) return st;
    if (reps < 1) reps = 1;
    char* ws = static_cast<char*>(workspace);
    // the costs (or row norms) do not depend on the schedule: compute them once
    st = run_front(*plan, X_packed, Y_packed, ws, stream);
    if (st != PARDTW_OK) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PARDTW_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PARDTW_ERR_HIP;
    }
    float best = INFINITY;
    int best_s = plan->chosen;
    for (size_t s = 0; s < plan->scheds.size() && st == PARDTW_OK; ++s) {
        const Schedule& sc = plan->scheds[s];
        st = run_dp(*plan, sc, ws, X_packed, Y_packed, totals, pair_status, stream);  // warm-up
        if (st != PARDTW_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) { st = PARDTW_ERR_HIP; break; }
        for (int r = 0; r < reps && st == PARDTW_OK; ++r)
            st = run_dp(*plan, sc, ws, X_packed, Y_packed, totals, pair_status, stream);
        if (st != PARDTW_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = PARDTW_ERR_HIP;
            break;
        }
        ms /= float(reps);
        if (ms < best) {
            best = ms;
            best_s = int(s);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PARDTW_OK) return st;
    plan->chosen = best_s;
    if (best_ms) *best_ms = best;
    return PARDTW_OK;
}

extern "C" pardtw_status pardtw_path_grad_batch(const pardtw_plan* plan, const float* X_packed,
                                                const float* Y_packed, const int32_t* paths_packed,
                                                const int32_t* path_len, const float* g_totals, float* dX_packed,
                                                float* dY_packed, hipStream_t stream) {
    if (!plan || !X_packed || !Y_packed || !paths_packed || !path_len || !g_totals || !dX_packed || !dY_packed)
        return PARDTW_ERR_INVALID_ARG;
    if (plan->mode != 0) return PARDTW_ERR_INVALID_ARG;
    return pardtw::grad_batch_launch(plan->pairs_dev, plan->batch, plan->max_cap, plan->d, X_packed, Y_packed,
                                     paths_packed, path_len, g_totals, dX_packed, plan->x_rows * plan->d,
                                     dY_packed, plan->y_rows * plan->d, stream);
}

// ---- Segmental DTW -----------------------------------------------------------

extern "C" pardtw_status pardtw_segplan_create(int64_t la, int64_t lb, int32_t nfrag, int64_t d, pardtw_prec prec,
                                               int32_t variant, int32_t flags, pardtw_plan** plan_out) {
    if (!plan_out) return PARDTW_ERR_INVALID_ARG;
    *plan_out = nullptr;
    if (nfrag <= 0 || la < nfrag || !pardtw::valid_sizes(la, lb) || d <= 0 || d > (int64_t(1) << 20))
        return PARDTW_ERR_INVALID_ARG;
    if (variant != PARDTW_NSDTW && variant != PARDTW_WSDTW) return PARDTW_ERR_INVALID_ARG;
    if (prec != PARDTW_PREC_F32 && prec != PARDTW_PREC_BF16) return PARDTW_ERR_UNSUPPORTED;
    if (!pardtw::valid_sizes(nfrag, lb)) return PARDTW_ERR_INVALID_ARG;
    if (const pardtw_status fs = check_flags(flags, d, prec); fs != PARDTW_OK) return fs;

    pardtw_plan* pl = new (std::nothrow) pardtw_plan;
    if (!pl) return PARDTW_ERR_HIP;
    pl->mode = 1;
    pl->variant = variant;
    pl->la = la;
    pl->lb = lb;
    pl->hop = std::max<int64_t>(1, la / (2 * int64_t(nfrag)));
    pl->batch = nfrag;
    pl->d = d;
    pl->prec = prec;
    pl->fused = (flags & PARDTW_PLAN_FUSED_COST) != 0;
    if (hipGetDevice(&pl->device) != hipSuccess ||
        hipDeviceGetAttribute(&pl->cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess) {
        delete pl;
        return PARDTW_ERR_HIP;
    }
    // fragment f: rows [floor(f la / N), floor((f+1) la / N)) of A against all of B
    pl->pairs.resize(nfrag);
    size_t c_floats = 0, bp_bytes = 0, rec_bytes = 0, rx_total = 0;
    int64_t tiles = 0;
    for (int f = 0; f < nfrag; ++f) {
        pardtw::BatchPair& q = pl->pairs[f];
        const int64_t r0 = int64_t(f) * la / nfrag, r1 = int64_t(f + 1) * la / nfrag;
        q.x_off = r0;
        q.y_off = 0;
        q.path_off = r0;  // fragment f's path slot: n_f pairs
        place_pair(q, r1 - r0, lb, pardtw::subseq_feasible(r1 - r0, lb), 2, pl->fused, c_floats, bp_bytes, rec_bytes,
                   rx_total, tiles);
        pl->max_cap = std::max(pl->max_cap, r1 - r0);
        pl->max_n = std::max(pl->max_n, r1 - r0);
    }
    pl->x_rows = la;
    pl->y_rows = lb;
    pl->path_capacity = la;
    pl->tiles = tiles;
    // cost panels | codes | DP header + records | scores | fragment statuses |
    // fragment path slots | fragment path lengths | segment-level workspace
    pl->off_c = 0;
    pl->off_rx = 0;
    pl->off_bp = align_up((pl->fused ? rx_total : c_floats) * sizeof(float));
    pl->off_dp = pl->off_bp + align_up(bp_bytes);
    pl->off_s = pl->off_dp + align_up(pardtw::dp_header_bytes() + rec_bytes);
    pl->off_fstat = pl->off_s + align_up(size_t(nfrag) * size_t(lb) * sizeof(float));
    pl->off_slots = pl->off_fstat + align_up(size_t(nfrag) * sizeof(int32_t));
    pl->off_flen = pl->off_slots + align_up(size_t(la) * 2 * sizeof(int32_t));
    pl->off_seg = pl->off_flen + align_up(size_t(nfrag) * sizeof(int32_t));
    // fragments of more than two segments get the split walk, as subsequence
    // paths from their ends
    int64_t nrec = 0, ncells = 0;
    for (int f = 0; f < nfrag; ++f) {
        pardtw::BatchPair& q = pl->pairs[f];
        int R, S;
        pardtw::split_shape(q.n, R, S);
        if (!q.feasible || S <= 2) continue;
        q.split = 1;
        const int32_t idx = int32_t(pl->segpairs.size());
        pl->segpairs.push_back({f, R, S, int32_t(pl->seg_map.size()), nrec, ncells});
        pl->seg_map.insert(pl->seg_map.end(), size_t(S), idx);
        nrec += 2 * int64_t(S);
        ncells += int64_t(S) * R * 2;
    }
    pl->off_split_rec = pl->off_seg + align_up(pardtw::segment_workspace_bytes_impl(nfrag, lb));
    pl->off_split_cells = pl->off_split_rec + align_up(size_t(nrec) * pardtw::split_record_bytes());
    pl->ws_bytes = pl->off_split_cells + align_up(size_t(ncells) * sizeof(int32_t));
    return finish_plan(pl, plan_out);
}

extern "C" int64_t pardtw_segplan_scores_offset(const pardtw_plan* plan) {
    return plan && plan->mode == 1 ? int64_t(plan->off_s) : -1;
}

extern "C" int64_t pardtw_segplan_hop(const pardtw_plan* plan) {
    return plan && plan->mode == 1 ? plan->hop : -1;
}

extern "C" int64_t pardtw_segplan_fragment_start(const pardtw_plan* plan, int32_t f) {
    if (!plan || plan->mode != 1 || f < 0 || f > plan->batch) return -1;
    return f == plan->batch ? plan->la : plan->pairs[f].x_off;
}

namespace {

pardtw_status check_seg_call(const pardtw_plan* plan, const float* A, const float* B, void* ws, size_t ws_bytes) {
    if (!plan || plan->mode != 1 || !A || !B || !ws) return PARDTW_ERR_INVALID_ARG;
    if (!aligned(ws, kAlign)) return PARDTW_ERR_INVALID_ARG;
    if (ws_bytes < plan->ws_bytes) return PARDTW_ERR_WORKSPACE;
    return PARDTW_OK;
}

pardtw_status seg_front(const pardtw_plan* plan, const float* A, const float* B, char* ws, hipStream_t stream) {
    pardtw_status st = pardtw::segment_init_launch(plan->pairs_dev, plan->batch,
                                                   reinterpret_cast<float*>(ws + plan->off_s),
                                                   reinterpret_cast<int32_t*>(ws + plan->off_fstat), stream);
    if (st != PARDTW_OK) return st;
    return run_front(*plan, A, B, ws, stream);
}

}  // namespace

extern "C" pardtw_status pardtw_segmental_align(const pardtw_plan* plan, const float* A, const float* B,
                                                void* workspace, size_t workspace_bytes, float* total, int32_t* ends,
                                                int32_t* path, int32_t* path_len, int32_t* status,
                                                hipStream_t stream) {
    pardtw_status st = check_seg_call(plan, A, B, workspace, workspace_bytes);
    if (st != PARDTW_OK) return st;
    if (!total || !ends || !path || !path_len || !status || !aligned(path, 8)) return PARDTW_ERR_INVALID_ARG;
    char* ws = static_cast<char*>(workspace);
    if ((st = seg_front(plan, A, B, ws, stream)) != PARDTW_OK) return st;
    if ((st = run_dp(*plan, plan->scheds[plan->chosen], ws, A, B, nullptr, nullptr, stream)) != PARDTW_OK) return st;
    st = pardtw::segment_ends_launch(reinterpret_cast<const float*>(ws + plan->off_s), plan->batch, plan->lb,
                                     plan->hop, plan->variant, ws + plan->off_seg, ends, total, status, stream);
    if (st != PARDTW_OK) return st;
    int32_t* slots = reinterpret_cast<int32_t*>(ws + plan->off_slots);
    int32_t* flen = reinterpret_cast<int32_t*>(ws + plan->off_flen);
    const uint8_t* bp = reinterpret_cast<const uint8_t*>(ws + plan->off_bp);
    st = pardtw::subseq_backtrace_batch_launch(plan->pairs_dev, plan->batch, bp, ends, slots, flen, stream);
    if (st != PARDTW_OK) return st;
    st = pardtw::split_backtrace_batch_launch(plan->pairs_dev, plan->segpairs_dev, int32_t(plan->segpairs.size()),
                                              plan->seg_map_dev, int32_t(plan->seg_map.size()), bp, nullptr, ends,
                                              ws + plan->off_split_rec,
                                              reinterpret_cast<int32_t*>(ws + plan->off_split_cells), slots, flen,
                                              stream);
    if (st != PARDTW_OK) return st;
    return pardtw::segment_gather_launch(plan->pairs_dev, plan->batch, slots, flen, status, path, path_len, stream);
}

extern "C" pardtw_status pardtw_segplan_autotune(pardtw_plan* plan, const float* A, const float* B,
                                                 void* workspace, size_t workspace_bytes, int32_t reps,
                                                 float* best_ms, hipStream_t stream) {
    pardtw_status st = check_seg_call(plan, A, B, workspace, workspace_bytes);
    if (st != PARDTW_OK) return st;
    if (reps < 1) reps = 1;
    char* ws = static_cast<char*>(workspace);
    if ((st = seg_front(plan, A, B, ws, stream)) != PARDTW_OK) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PARDTW_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PARDTW_ERR_HIP;
    }
    float best = INFINITY;
    int best_s = plan->chosen;
    for (size_t s = 0; s < plan->scheds.size() && st == PARDTW_OK; ++s) {
        const Schedule& sc = plan->scheds[s];
        st = run_dp(*plan, sc, ws, A, B, nullptr, nullptr, stream);  // warm-up
        if (st != PARDTW_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) { st = PARDTW_ERR_HIP; break; }
        for (int r = 0; r < reps && st == PARDTW_OK; ++r) st = run_dp(*plan, sc, ws, A, B, nullptr, nullptr, stream);
        if (st != PARDTW_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = PARDTW_ERR_HIP;
            break;
        }
        ms /= float(reps);
        if (ms < best) {
            best = ms;
            best_s = int(s);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PARDTW_OK) return st;
    plan->chosen = best_s;
    if (best_ms) *best_ms = best;
    return PARDTW_OK;
}
