// Deferred placement of a plain DFA scan's matches.
//
// In a plain scan (one input, no carried instances, output from offset 0)
// of at least kDeferMinSegs segments, a segment whose matches fit its LDS
// buffer does not wait in the look-back for its output offset.  It ranks its
// matches, writes them to a staging area at rows it claims from a counter,
// publishes its count and takes its next segment.  A follow-up launch on the
// same stream then sums the counts before each segment and copies its staged
// rows into place (above kDeferFusedSegs segments, two launches: a scan of
// the counts, then the copy).  A segment whose matches did not fit its
// buffer, or that finds the staging area full, is placed by the scan kernel
// as before; the counts it sums in the look-back are the ones every segment
// publishes before it moves on.  Batches and streams place every segment in
// the scan.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "pfsm_dev.h"

namespace pfsmk {

struct DfaDefer {
    MatchOut *stage;             // staged rows; NULL: every segment is placed by the scan
    int64_t stage_cap;           // rows the scan may claim
    unsigned long long *cursor;  // rows claimed so far (cleared by the offset scan)
    long long *seg_at;           // [n_segs] first staged row, -1: placed by the scan
    long long *seg_cnt;          // [n_segs] matches of the segment
    long long *seg_base;         // [n_segs] output offset (exclusive scan of seg_cnt)
};

constexpr int64_t kDeferRowsMax = 4ll << 20;  // staging rows kept per workspace at most
constexpr int kDeferFusedSegs = 4096;         // up to this many segments: one follow-up launch
// Fewer segments than this are placed by the scan itself: their waits are
// short, and a follow-up launch would add to a small scan's latency.
constexpr int kDeferMinSegs = 64;

// The follow-up launches of a deferred scan of n_segs (>= 1) segments:
// offsets and *total, and the copy of staged rows below `cap` into `out`.
hipError_t launch_dfa_place(const DfaDefer &d, int n_segs, int64_t *total, MatchOut *out, int64_t cap,
                            hipStream_t s);

}  // namespace pfsmk
