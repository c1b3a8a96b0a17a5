// Device helpers shared by the scan kernels: wave64 compaction, block
// reductions and the decoupled look-back that turns per-window match counts
// into global output offsets in a single pass.
#pragma once

#include "pfsm_dev.h"

namespace pfsmk {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Reserve one slot per lane with `pred` in an LDS queue: one LDS atomic per
// wave, ranks from the ballot's prefix popcount.  Returns -1 when !pred.
__device__ __forceinline__ int wave_reserve(int *counter, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    return pred ? base + rank : -1;
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Inclusive scan across a wave64.
__device__ __forceinline__ long long wave_incl_scan(long long v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        long long t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Sum of `v` over the block; every thread gets the result.  `red` holds
// kBlock/64 slots.  Contains two barriers.
__device__ __forceinline__ long long block_sum(long long v, long long *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Exclusive scan of `v` over the block in thread order; *total receives the
// sum.  `red` holds kBlock/64 slots.  Contains two barriers.
__device__ __forceinline__ long long block_excl_scan(long long v, long long *red, long long *total) {
    const long long inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) red[w] = inc;
    __syncthreads();
    long long before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) before += red[i];
        all += red[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ unsigned long long status_load(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void status_store(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back, run by one whole wave for window `w` whose own count
// is `mine`.  Publishes the aggregate, walks predecessors 64 at a time until
// an inclusive prefix is found, publishes its own inclusive prefix and
// returns the exclusive prefix (in every lane).  Windows are numbered in
// ticket order, so every predecessor is already running and publishes its
// aggregate without waiting on anyone: the spin always ends.
__device__ __forceinline__ long long lookback(unsigned long long *status, long long w, long long mine) {
    const int lane = lane_id();
    if (w == 0) {
        if (lane == 0) status_store(&status[0], kStatPre | (unsigned long long)mine);
        return 0;
    }
    if (lane == 0) status_store(&status[w], kStatAgg | (unsigned long long)mine);
    long long excl = 0;
    long long look = w - 1;
    for (;;) {
        const long long idx = look - lane;
        unsigned long long v = idx >= 0 ? status_load(&status[idx]) : kStatPre;
        while (__any((v >> 62) == 0)) {
            __builtin_amdgcn_s_sleep(1);
            if ((v >> 62) == 0) v = status_load(&status[idx]);
        }
        const unsigned long long pm = __ballot((v >> 62) == 2);
        const long long val = (long long)(v & kStatVal);
        if (pm) {
            const int j = __ffsll((long long)pm) - 1;
            excl += wave_sum(lane <= j ? val : 0);
            break;
        }
        excl += wave_sum(val);
        look -= 64;
    }
    if (lane == 0) status_store(&status[w], kStatPre | (unsigned long long)(excl + mine));
    return excl;
}

// End-of-launch bookkeeping: add this block's counters, and let the last
// block to finish publish the launch's totals and reset the control block and
// the status words for the next launch.  Call from every thread.
__device__ __forceinline__ void finish_launch(ScanCtl *ctl, unsigned long long *status, int n_windows,
                                              long long T, long long X, long long L, long long M,
                                              int *last_flag) {
    if (threadIdx.x == 0) {
        if (T) atomicAdd(&ctl->acc[0], (unsigned long long)T);
        if (X) atomicAdd(&ctl->acc[1], (unsigned long long)X);
        if (L) atomicAdd(&ctl->acc[2], (unsigned long long)L);
        if (M) atomicAdd(&ctl->acc[3], (unsigned long long)M);
        __threadfence();
        const unsigned prev = atomicAdd(&ctl->done, 1u);
        *last_flag = (prev == (unsigned)(n_windows - 1));
    }
    __syncthreads();
    if (*last_flag) {
        __threadfence();
        for (int i = threadIdx.x; i < n_windows; i += kBlock) status[i] = 0;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) ctl->last[k] = (long long)atomicExch(&ctl->acc[k], 0ull);
            ctl->ticket = 0;
            ctl->done = 0;
        }
    }
}

// Stage x[0, len) into LDS (len <= capacity), 16 bytes per load when the
// source is 16-byte aligned.
__device__ __forceinline__ void stage_bytes(uint8_t *dst, const uint8_t *src, int len) {
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const int nv = len >> 4;
        const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
        uint4 *d4 = reinterpret_cast<uint4 *>(dst);
        for (int c = threadIdx.x; c < nv; c += kBlock) d4[c] = s4[c];
        for (int i = (nv << 4) + threadIdx.x; i < len; i += kBlock) dst[i] = src[i];
    } else {
        for (int i = threadIdx.x; i < len; i += kBlock) dst[i] = src[i];
    }
}

}  // namespace pfsmk
