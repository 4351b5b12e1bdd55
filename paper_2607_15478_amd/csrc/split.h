// The split walk: a backtrace cut into segments of rows that many workgroups
// walk at once, then joined exactly (the serial walk of Sec. II-D's backtrace
// matrix, or of its checkpointed form, gives the same path).
//
// Segment s of S holds the path's cells on rows (s R - 1, (s + 1) R - 1]
// (segment 0 down to the origin, or for a subsequence path (Sec. II-B) down to
// its start on row 0). It starts at the first path cell on or below its top
// row, which is where the segment above ends (a step moves at most two rows,
// so every segment holds at least one cell).
//   round 0: every segment walks from a guess on its top row (DTW: the
//            diagonal through the corners, clamped to the band; subsequence:
//            the line of slope one into the end, clamped to the cells that
//            row 0 reaches and that reach the end); the last segment starts
//            exactly, at (n-1, m-1) or (n-1, end);
//   round r: every segment walks again from where the segment above ended in
//            round r - 1, unless it already started there;
//   finish:  one workgroup checks, from the last segment down, that each
//            segment started where the one above ended, and walks again any
//            that did not (its start is then exact); then it takes the
//            offsets and the length, and a copy lays the segments out in
//            forward order.
// Whatever the guesses, every segment is at last walked from its exact start,
// so the path is the serial walk's; good guesses only save the serial rewalks.
// Optimal paths walked back from nearby cells merge within a few dozen steps,
// so after round 1 the starts are nearly always exact.
#pragma once

#include "common.h"

namespace pardtw {
namespace {

struct SegInfo {
    int32_t si, sj;  // start cell
    int32_t ei, ej;  // first cell past the segment (segment 0: unused)
    int32_t len;     // cells written (0: the walk failed)
    int32_t off;     // position of the segment's last cell in the path
    int32_t pad[2];
};

constexpr int kSegMaxCount = 256;  // segments of one walk at most

struct SplitArgs {
    int n, m;
    int end;  // the path's last column: m - 1 for DTW, the chosen end for a subsequence path
    int sub;  // nonzero: a subsequence path, walked back to row 0
    int R, S;
    SegInfo* info;   // [2][S]: rounds alternate between the halves
    int32_t* cells;  // [S][R][2]: segment s's cells from its start backward
};

__host__ __device__ inline int seg_stop_row(int s, int R) { return s == 0 ? -1 : s * R - 1; }

// A cell on row i of the band (reachable from the origin, reaching (n-1, m-1))
// near the diagonal through the corners.
__device__ inline int seg_guess_col(int i, int n, int m) {
    const int64_t jd = (int64_t(i) * (m - 1) + (n - 1) / 2) / (n > 1 ? n - 1 : 1);
    const int64_t lo1 = (i + 1) / 2, lo2 = int64_t(m - 1) - 2 * int64_t(n - 1 - i);
    const int64_t hi1 = 2 * int64_t(i), hi2 = int64_t(m - 1) - (int64_t(n - 1 - i) + 1) / 2;
    const int64_t lo = lo1 > lo2 ? lo1 : lo2, hi = hi1 < hi2 ? hi1 : hi2;
    const int64_t c = jd < lo ? lo : jd > hi ? hi : jd;
    return int(c < 0 ? 0 : c > m - 1 ? m - 1 : c);
}

// A guess on row i for a subsequence path ending at (n-1, end): the line of
// slope one into the end, clamped to the cells that row 0 reaches (at least
// ceil(i/2) columns in) and that reach the end (1 to 2 columns per row).
__device__ inline int seg_guess_col_sub(int i, int n, int end) {
    const int64_t di = int64_t(n - 1 - i);
    const int64_t lo1 = (i + 1) / 2, lo2 = int64_t(end) - 2 * di;
    const int64_t hi = int64_t(end) - (di + 1) / 2;
    const int64_t lo = lo1 > lo2 ? lo1 : lo2;
    int64_t c = int64_t(end) - di;
    c = c < lo ? lo : c;
    c = c > hi ? hi : c;
    return int(c < 0 ? 0 : c > end ? end : c);
}

__device__ inline SegInfo seg_info(int si, int sj, int ei, int ej, int len) {
    SegInfo r;
    r.si = si;
    r.sj = sj;
    r.ei = ei;
    r.ej = ej;
    r.len = len;
    r.off = 0;
    r.pad[0] = r.pad[1] = 0;
    return r;
}

// One round for segment s. walk(s, si, sj, out) walks segment s from (si, sj)
// with the whole workgroup, writes its cells at a.cells + s R 2 and its
// record to *out, and returns the record to every thread.
template <class Walk>
__device__ void split_round(const SplitArgs& a, int s, int round, Walk&& walk) {
    const SegInfo* prev = a.info + (round & 1 ? 0 : a.S);
    SegInfo* cur = a.info + (round & 1 ? a.S : 0);
    int si, sj;
    if (s == a.S - 1) {
        si = a.n - 1;
        sj = a.end;
    } else if (round == 0) {
        si = (s + 1) * a.R - 1;
        sj = a.sub ? seg_guess_col_sub(si, a.n, a.end) : seg_guess_col(si, a.n, a.m);
    } else {
        const SegInfo up = prev[s + 1];
        si = up.ei;
        sj = up.ej;
    }
    if (round > 0) {
        const SegInfo me = prev[s];
        // unchanged start (or none known: the segment above failed)
        if ((me.si == si && me.sj == sj && me.len > 0) || si < 0) {
            if (threadIdx.x == 0) cur[s] = me;
            return;
        }
    }
    walk(s, si, sj, cur + s);
}

// The check from the last segment down (`fin`: the half the last round
// wrote); sinfo holds kSegMaxCount records in LDS.
template <class Walk>
__device__ void split_finish(const SplitArgs& a, SegInfo* sinfo, int fin, int cap, int32_t* path_len, Walk&& walk) {
    const int tid = threadIdx.x;
    SegInfo* info = a.info + fin * a.S;
    for (int k = tid; k < a.S; k += int(blockDim.x)) sinfo[k] = info[k];
    __syncthreads();
    int si = a.n - 1, sj = a.end;
    for (int s = a.S - 1; s >= 0; --s) {
        SegInfo me = sinfo[s];
        if (me.si != si || me.sj != sj || me.len <= 0) {
            me = walk(s, si, sj, info + s);
            if (me.len <= 0) {
                if (tid == 0) *path_len = 0;
                return;
            }
            if (tid == 0) sinfo[s] = me;
        }
        si = me.ei;
        sj = me.ej;
    }
    // offsets: segment s's cells go after those of segments 0 .. s-1
    if (tid == 0) {
        int64_t off = 0;
        for (int s = 0; s < a.S; ++s) {
            info[s].off = int32_t(off);
            off += sinfo[s].len;
        }
        *path_len = off > cap ? 0 : int32_t(off);
    }
}

// Copies segment s, reversed, to its place in the path.
__device__ inline void split_copy(const SplitArgs& a, int s, int fin, int32_t* path) {
    const SegInfo me = a.info[fin * a.S + s];
    const int2* src = reinterpret_cast<const int2*>(a.cells + int64_t(s) * a.R * 2);
    int2* dst = reinterpret_cast<int2*>(path) + me.off;
    for (int k = threadIdx.x; k < me.len; k += blockDim.x) dst[me.len - 1 - k] = src[k];
}

}  // namespace
}  // namespace pardtw
