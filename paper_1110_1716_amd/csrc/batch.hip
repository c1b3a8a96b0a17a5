// Planning and gathering kernels of a batched scan: many byte streams, each
// scanned against one of several resident automata (the union model of
// Section III.A applied per stream).  All bookkeeping stays on the device,
// so a batch needs no host round trip before its scan launches.
//
//   plan    one workgroup: per stream, the number of segments; per automaton,
//           an exclusive scan of those counts in stream order (each stream's
//           first segment within its automaton's launch), the automaton's
//           segment count and the offset of its list.
//   fill    one thread per stream: writes the stream index of every one of
//           its segments into its automaton's list.
//   (the scan kernels: one launch per automaton; each writes its matches
//    after the previous automaton's, and each stream's output range)
//   offsets one workgroup: exclusive scan of the per-stream counts into the
//           caller's group offsets.
//   gather  every output position takes its match from the stage (binary
//           search of the position's stream).
#include "batch.h"
#include "scan_common.h"

namespace pfsmk {

namespace {

constexpr int PT = 1024;

__global__ __launch_bounds__(PT) void batch_plan_kernel(BatchPlanArgs p) {
    __shared__ int run[kMaxBatchAutomata];
    __shared__ long long bytes_s[kMaxBatchAutomata];
    __shared__ long long seg_s[kMaxBatchAutomata];
    __shared__ long long red[PT / 64];
    __shared__ int err_s;
    const int tid = threadIdx.x;
    if (tid < p.n_aut) {
        run[tid] = 0;
        bytes_s[tid] = 0;
    }
    if (tid == 0) err_s = 0;
    __syncthreads();
    // Pass 1: validate, clear the stream ranges, sum the bytes per automaton.
    for (int c0 = 0; c0 < p.n_streams; c0 += PT) {
        const int s = c0 + tid;
        int aut = -1;
        int64_t len = 0;
        if (s < p.n_streams) {
            aut = p.stream_aut[s];
            len = p.stream_off[s + 1] - p.stream_off[s];
            if (aut < 0 || aut >= p.n_aut) err_s = 1;
            if (len < 0 || len > p.max_stream) err_s = 2;
            p.stream_lo[s] = 0;
            p.stream_hi[s] = 0;
        }
        for (int a = 0; a < p.n_aut; ++a) {
            const long long t = block_sum<PT>(aut == a && len > 0 ? len : 0, red);
            if (tid == 0) bytes_s[a] += t;
        }
    }
    __syncthreads();
    // Segment size of each launch: its bytes over about twice its resident
    // workgroups, within [seg_min, seg_max], a multiple of 16 (or the size
    // set for the automaton).
    if (tid < p.n_aut) {
        const long long want = 2ll * (p.blocks[tid] > 0 ? p.blocks[tid] : 1);
        long long sg = (bytes_s[tid] + want - 1) / want;
        sg = (sg + 15) / 16 * 16;
        sg = sg < p.seg_min ? p.seg_min : (sg > p.seg_max ? p.seg_max : sg);
        if (p.seg_fix[tid] > 0) sg = p.seg_fix[tid];
        seg_s[tid] = sg;
        p.seg[tid] = sg;
    }
    __syncthreads();
    // Pass 2: segments per stream, scanned per automaton in stream order.
    for (int c0 = 0; c0 < p.n_streams; c0 += PT) {
        const int s = c0 + tid;
        const bool valid = s < p.n_streams;
        const int aut = valid ? p.stream_aut[s] : -1;
        const int64_t len = valid ? p.stream_off[s + 1] - p.stream_off[s] : 0;
        const bool ok = valid && aut >= 0 && aut < p.n_aut && len > 0 && len <= p.max_stream;
        const long long nseg = ok ? (len + seg_s[aut] - 1) / seg_s[aut] : 0;
        for (int a = 0; a < p.n_aut; ++a) {
            long long tot;
            const long long ex = block_excl_scan<PT>(aut == a ? nseg : 0, red, &tot);
            if (ok && aut == a) p.seg_first[s] = (int32_t)(run[a] + ex);
            __syncthreads();
            if (tid == 0) run[a] += (int)tot;
            __syncthreads();
        }
    }
    __syncthreads();
    if (tid == 0) {
        int total = 0, mx = 0;
        for (int a = 0; a < p.n_aut; ++a) {
            p.seg_base[a] = total;
            total += run[a];
            mx = run[a] > mx ? run[a] : mx;
        }
        p.info->err = err_s;
        p.info->total_segs = total;
        p.info->max_segs = mx;
        p.bases[0] = 0;
        // Nothing is scanned when the plan does not fit: the host grows the
        // buffers and plans again.
        const bool runnable = err_s == 0 && total <= p.seg_cap && mx <= p.lb_cap;
        for (int a = 0; a < p.n_aut; ++a) p.n_segs[a] = runnable ? run[a] : 0;
    }
}

__global__ void batch_fill_kernel(BatchPlanArgs p) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_streams) return;
    if (p.info->err || p.info->total_segs > p.seg_cap || p.info->max_segs > p.lb_cap) return;
    const int aut = p.stream_aut[s];
    const int64_t len = p.stream_off[s + 1] - p.stream_off[s];
    if (len <= 0) return;
    const int nseg = (int)((len + p.seg[aut] - 1) / p.seg[aut]);
    const int base = p.seg_base[aut] + p.seg_first[s];
    for (int j = 0; j < nseg; ++j) p.seg_stream[base + j] = s;
}

__global__ __launch_bounds__(PT) void batch_offsets_kernel(BatchGatherArgs g) {
    __shared__ long long red[PT / 64];
    const int tid = threadIdx.x;
    long long run = 0;
    for (int c0 = 0; c0 < g.n_streams; c0 += PT) {
        const int s = c0 + tid;
        const long long cnt = s < g.n_streams ? g.stream_hi[s] - g.stream_lo[s] : 0;
        long long tot;
        const long long ex = block_excl_scan<PT>(cnt, red, &tot);
        if (s < g.n_streams) g.match_off[s] = run + ex;
        run += tot;
    }
    if (tid == 0) {
        g.match_off[g.n_streams] = run;
        g.info->total = run;
    }
}

__global__ void batch_gather_kernel(BatchGatherArgs g) {
    const int64_t total = g.info->total;
    const int64_t lim = total < g.cap ? total : g.cap;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < lim; o += (int64_t)gridDim.x * blockDim.x) {
        // the stream whose group holds position o: last s with match_off[s] <= o
        int lo = 0, hi = g.n_streams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g.match_off[mid] <= o) lo = mid;
            else hi = mid - 1;
        }
        const int64_t src = g.stream_lo[lo] + (o - g.match_off[lo]);
        if (src < g.stage_cap) g.out[o] = g.stage[src];
    }
}

}  // namespace

hipError_t launch_batch_plan(const BatchPlanArgs &p, hipStream_t s) {
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(PT), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.n_streams == 0) return e;
    hipLaunchKernelGGL(batch_fill_kernel, dim3((p.n_streams + 255) / 256), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchGatherArgs &g, hipStream_t s) {
    hipLaunchKernelGGL(batch_offsets_kernel, dim3(1), dim3(PT), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_gather_kernel, dim3(1024), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace pfsmk
