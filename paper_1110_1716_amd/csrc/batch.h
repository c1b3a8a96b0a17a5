// Batched scans: argument blocks of the planning and gathering kernels
// (internal to libpfsm).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfsm_dev.h"

namespace pfsmk {

constexpr int kMaxBatchAutomata = 64;
constexpr int64_t kBatchSeg = 65536;  // bytes per segment (both scan kernels)

// What the device reports back about a batch.
struct BatchInfo {
    int32_t err;         // 1: an automaton index out of range, 2: a bad stream length
    int32_t total_segs;  // segments over all automata
    int32_t max_segs;    // segments of the largest launch
    int32_t pad;
    int64_t total;       // matches over all streams
};

struct BatchPlanArgs {
    const int64_t *stream_off;  // [n_streams + 1]
    const int32_t *stream_aut;  // [n_streams]
    int32_t n_streams, n_aut;
    int64_t seg, max_stream;
    int32_t *seg_first;         // [n_streams]
    int32_t *seg_stream;        // [seg_cap]
    int32_t *n_segs;            // [n_aut]
    int32_t *seg_base;          // [n_aut]
    int64_t *bases;             // [n_aut + 1] output index of each launch's first match
    int64_t *stream_lo, *stream_hi;  // [n_streams]
    BatchInfo *info;
    int32_t seg_cap, lb_cap;
};

struct BatchGatherArgs {
    int32_t n_streams;
    const int64_t *stream_lo, *stream_hi;
    int64_t *match_off;         // [n_streams + 1] (the caller's)
    const MatchOut *stage;
    int64_t stage_cap;
    MatchOut *out;              // the caller's
    int64_t cap;
    BatchInfo *info;
};

hipError_t launch_batch_plan(const BatchPlanArgs &p, hipStream_t s);
hipError_t launch_batch_gather(const BatchGatherArgs &g, hipStream_t s);

}  // namespace pfsmk
