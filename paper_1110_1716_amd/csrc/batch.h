// Batched scans: argument blocks of the planning and gathering kernels
// (internal to libpfsm).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pfsm_dev.h"

struct pfsm;

namespace pfsmk {

struct Workspace;

constexpr int kMaxBatchAutomata = 64;
constexpr int64_t kBatchSegMax = 65536;  // bytes per segment (both scan kernels)
constexpr int64_t kBatchSegMin = 4096;

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
    int64_t seg_min, seg_max, max_stream;
    int32_t *seg_first;         // [n_streams]
    int32_t *seg_stream;        // [seg_cap]
    int32_t *n_segs;            // [n_aut]
    int32_t *seg_base;          // [n_aut]
    int64_t *bases;             // [n_aut + 1] output index of each launch's first match
    int64_t *seg;               // [n_aut] bytes per segment of each launch
    int32_t blocks[kMaxBatchAutomata];  // resident workgroups of each launch's kernel
    int32_t seg_fix[kMaxBatchAutomata]; // bytes per segment chosen for the automaton, 0 = adaptive
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

// A batch enqueued by batch_run: what the device reports about it is in
// *info (device memory) once the stream has reached the batch's end.
struct BatchRun {
    BatchInfo *info = nullptr;
    const int64_t *stream_lo = nullptr;  // each stream's range in the stage
    const int64_t *stream_hi = nullptr;
    int64_t stage_cap = 0;
    int32_t seg_cap = 0;
    int lb_cap = 0;
    std::vector<struct Workspace *> ws;
    void *bw = nullptr;
};

// Enqueue a whole batch on s (buffers grown first, which may synchronise s).
int batch_run(struct ::pfsm *const *hs, int32_t n_automata, const uint8_t *d_data, const int64_t *d_stream_off,
              const int32_t *d_stream_automaton, int32_t n_streams, MatchOut *d_out, int64_t cap,
              int64_t *d_match_off, hipStream_t s, BatchRun *run);
// After a batch whose plan did not fit (info.total_segs > seg_cap or
// info.max_segs > lb_cap): grow what it needs.  Returns true in *again when
// the batch must be enqueued again.
int batch_fit(BatchRun *run, const BatchInfo &info, hipStream_t s, bool *again);

}  // namespace pfsmk
