// Device helpers shared by the scan kernels: wave64 compaction, block
// reductions, 16-byte input loads and the cross-workgroup prefix that turns
// per-workgroup match counts into output offsets.
#pragma once

#include "pfsm_dev.h"

namespace pfsmk {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long lanes_below() {
    return (1ull << lane_id()) - 1ull;
}

// Set bits of m in the lanes below this one (two mbcnt instructions).
__device__ __forceinline__ int lanes_below_count(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Reserve one slot per lane with `pred` in a wave-private LDS queue whose
// count lives in a wave-uniform register.  Returns the slot or -1.
__device__ __forceinline__ int wave_push_slot(int &count, bool pred) {
    const unsigned long long m = __ballot(pred);
    const int slot = count + lanes_below_count(m);
    count += __popcll(m);
    return pred ? slot : -1;
}

// Exclusive prefix over the wave of a count in [0, 16), and the wave total.
__device__ __forceinline__ int wave_excl_small(int v, int &total) {
    int ex = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        const unsigned long long m = __ballot((v >> bit) & 1);
        ex += lanes_below_count(m) << bit;
        tot += __popcll(m) << bit;
    }
    total = tot;
    return ex;
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

// Sum of `v` over a block of NT threads; every thread gets the result.
// `red` holds NT/64 slots.  Contains two barriers.
template <int NT>
__device__ __forceinline__ long long block_sum(long long v, long long *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    long long s = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Sums of four values over a block of NT threads (every thread gets them).
// `red` holds 4 * NT/64 slots.  Contains two barriers.
template <int NT>
__device__ __forceinline__ void block_sum4(long long v[4], long long *red) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long s = wave_sum(v[k]);
        if (lane_id() == 0) red[4 * w + k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        long long s = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += red[4 * i + k];
        v[k] = s;
    }
    __syncthreads();
}

// Exclusive scan of `v` over a block of NT threads in thread order; *total
// receives the sum.  `red` holds NT/64 slots.  Contains two barriers.
template <int NT>
__device__ __forceinline__ long long block_excl_scan(long long v, long long *red, long long *total) {
    const long long inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) red[w] = inc;
    __syncthreads();
    long long before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        if (i < w) before += red[i];
        all += red[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ unsigned long long slot_load(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void slot_store(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The epoch this launch starts with: one past the epoch of the workgroup's
// own slot (every slot carries the same epoch between launches).
__device__ __forceinline__ unsigned first_epoch(const unsigned long long *slots, int b) {
    return (unsigned)((slot_load(&slots[b]) >> kEpochShift) + 1) & kEpochMask;
}

// Publish this workgroup's count for `epoch`, then read every peer's slot of
// the same epoch.  Returns the sum over lower-numbered workgroups; *round
// receives the sum over all of them.  Every workgroup of the grid is resident
// (cooperative launch) and publishes before it waits, so the waits end.
// Contains barriers; call from every thread.
template <int NT>
__device__ __forceinline__ long long grid_prefix(unsigned long long *slots, int nb, int b, unsigned epoch,
                                                 long long mine, long long *red, long long *round) {
    if (threadIdx.x == 0)
        slot_store(&slots[b], ((unsigned long long)epoch << kEpochShift) | (unsigned long long)mine);
    long long ex = 0, all = 0;
    for (int j = threadIdx.x; j < nb; j += NT) {
        long long c;
        if (j == b) {
            c = mine;
        } else {
            unsigned long long v = slot_load(&slots[j]);
            while (((unsigned)(v >> kEpochShift) & kEpochMask) != epoch) {
                __builtin_amdgcn_s_sleep(1);
                v = slot_load(&slots[j]);
            }
            c = (long long)(v & kCountMask);
        }
        all += c;
        if (j < b) ex += c;
    }
    const long long e = block_sum<NT>(ex, red);
    *round = block_sum<NT>(all, red);
    return e;
}

__device__ __forceinline__ unsigned long long lb_pack(unsigned epoch, int status, long long v) {
    const unsigned long long u = v < 0 ? 0ull : ((unsigned long long)v > kLbValMask ? kLbValMask : (unsigned long long)v);
    return ((unsigned long long)epoch << kLbEpochShift) | ((unsigned long long)status << kLbStatShift) | u;
}

// The epoch of this launch's look-back words (never 0, the value of a
// cleared word).
__device__ __forceinline__ unsigned lb_epoch(const ScanCtl *ctl) {
    const unsigned e = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return e % kLbEpochMod + 1;
}

// Next segment for this workgroup (thread 0 only).
__device__ __forceinline__ int take_ticket(ScanCtl *ctl) {
    return (int)atomicAdd(&ctl->ticket, 1ull);
}

// Decoupled look-back over segments in ticket order, run by one whole wave
// once segment s has been scanned: publishes its count, sums the counts of
// its predecessors back to the nearest one that has published a prefix,
// publishes its own prefix and returns the sum before s (every lane).  The
// predecessors of s took their tickets before s did, so their workgroups are
// running, and each publishes its count before it looks back itself: the
// waits end whether or not the whole grid is resident.
__device__ __forceinline__ long long lookback(unsigned long long *lb, int s, unsigned epoch, long long agg) {
    const int lane = lane_id();
    if (s == 0) {
        if (lane == 0) slot_store(&lb[0], lb_pack(epoch, kLbIncl, agg));
        return 0;
    }
    if (lane == 0) slot_store(&lb[s], lb_pack(epoch, kLbAgg, agg));
    long long ex = 0;
    int hi = s - 1;
    for (;;) {
        const int j = hi - lane;  // lane 0 is the nearest predecessor
        int st = kLbIncl;
        long long v = 0;
        if (j >= 0) {
            const unsigned long long w = slot_load(&lb[j]);
            st = (unsigned)(w >> kLbEpochShift) == epoch ? (int)((w >> kLbStatShift) & 3u) : 0;
            v = (long long)(w & kLbValMask);
        }
        const unsigned long long m_inc = __ballot(st == kLbIncl);
        const unsigned long long m_none = __ballot(st == 0);
        if (m_inc) {
            const int k = __ffsll((long long)m_inc) - 1;
            const unsigned long long need = k == 63 ? ~0ull : ((2ull << k) - 1ull);
            if ((m_none & need) == 0) {
                ex += wave_sum(lane <= k ? v : 0);
                break;
            }
        } else if (m_none == 0) {
            ex += wave_sum(v);
            hi -= 64;
            continue;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) slot_store(&lb[s], lb_pack(epoch, kLbIncl, agg + ex));
    return ex;
}

// End of a workgroup's part of a launch (call from every thread; contains
// barriers).  The last workgroup to finish resets the ticket counter and
// advances the epoch; when the epoch is about to wrap it first clears the
// look-back words, so a word left from an earlier launch never carries the
// epoch in use.
template <int NT>
__device__ __forceinline__ void finish_launch(ScanCtl *ctl, unsigned long long *lb, int lb_cap, int *flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned d = atomicAdd(&ctl->done, 1u);
        *flag = d + 1 == gridDim.x;
    }
    __syncthreads();
    if (!*flag) return;
    __threadfence();
    const unsigned e = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool wrap = (e + 1) % kLbEpochMod == 0;
    if (wrap)
        for (int i = threadIdx.x; i < lb_cap; i += NT) slot_store(&lb[i], 0ull);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(&ctl->ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->epoch, wrap ? 0u : e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Segment sg of a launch: its stream's bytes (sx, sn), the stream position
// of its first start and its stream (-1 for a single-stream launch).
__device__ __forceinline__ void seg_resolve(const SegPlan &p, const uint8_t *x, int64_t n, int64_t seg, int sg,
                                            int seg_base, const uint8_t *&sx, int64_t &sn, int64_t &seg_lo,
                                            int &stream) {
    if (p.stream_off) {
        stream = p.seg_stream[seg_base + sg];
        const int64_t o0 = p.stream_off[stream], o1 = p.stream_off[stream + 1];
        sx = x + o0;
        sn = o1 - o0;
        seg_lo = (int64_t)(sg - p.seg_first[stream]) * seg;
    } else {
        stream = -1;
        sx = x;
        sn = n;
        seg_lo = (int64_t)sg * seg;
    }
}

// The 16-byte granule of a 16-byte aligned input starting at `pos` (a
// multiple of 16 below n).  Bytes at or past n are unspecified: callers never
// use them.  The granule holds at least one valid byte, so it lies on a page
// of the input and the load cannot fault.
__device__ __forceinline__ uint4 load_granule(const uint8_t *x, int64_t pos) {
    return *reinterpret_cast<const uint4 *>(x + pos);
}

__device__ __forceinline__ int byte_of(const uint4 &v, int k) {
    const uint32_t w = k < 4 ? v.x : k < 8 ? v.y : k < 12 ? v.z : v.w;
    return (int)((w >> (8 * (k & 3))) & 0xffu);
}

}  // namespace pfsmk
