// Tag-merged DFA scan for gfx950 (Section III.B: an active state carries the
// set of tags of the instances in it, and tags move with their state).
//
// Instances in the same state at the same position have the same future, so
// they can take their transitions together.  One wave owns the starts of a
// segment and steps through the input one byte at a time from the
// segment's first start until all of its instances have died:
//   * every distinct active state is an entry held by one lane (state, the
//     list of its tags, their number); a DFA with at most kMergedStates
//     states never needs more than one entry per lane;
//   * each step looks up one transition per entry, however many instances
//     the entry holds, and adds the instance started at the current byte
//     (while inside the segment) as a new entry in a free lane;
//   * entries whose targets coincide merge: one lane wins the target in an
//     LDS table, the others append their tag lists to its list through an
//     atomic exchange of the list tail (tag lists are linked through an LDS
//     array indexed by tag);
//   * an entry in a final state reports every label for every tag it holds.
// The wave walks its segment twice: a count pass records each tag's number
// of matches, an exclusive scan over the tags and a decoupled look-back over
// segments (in ticket order, as in the per-start scan) place them, and a
// write pass stores them, so each start's matches come out in (end, label)
// order and starts in increasing order.
//
// A step costs a handful of LDS round trips whatever the number of live
// instances, which pays when walks are long (an instance lives for many
// bytes) and states are few; the per-start scan stays the default.
#include "pfsm_dev.h"
#include "scan_common.h"

namespace pfsmk {

namespace {

constexpr int MT = kMergedThreads;
constexpr int MW = MT / 64;
constexpr int SEG = kMergedSeg;
constexpr int WIN = 1024;  // staged bytes per wave window (16 per lane)

__global__ __launch_bounds__(MT) void dfa_merged_kernel(MergedArgs a) {
    __shared__ uint8_t tab_s[kMergedStates * 256];
    __shared__ uint8_t flags_s[64];
    __shared__ int32_t laboff_s[65];
    __shared__ int16_t next_s[MW][SEG];   // tag list links (-1: end)
    __shared__ long long kc_s[MW][SEG];   // matches per tag, then output offsets
    __shared__ uint8_t stage_s[MW][WIN];
    __shared__ int32_t own_s[MW][64], tail_s[MW][64], size_s[MW][64];
    __shared__ long long red4[4 * MW];
    __shared__ unsigned epoch_s;
    __shared__ int last_s;

    const int tid = threadIdx.x;
    const int wv = tid >> 6;
    const int lane = lane_id();
    const int N = a.n_states;
    for (int i = tid; i < N * 256; i += MT) tab_s[i] = a.tab[i];
    for (int i = tid; i < N; i += MT) flags_s[i] = a.flags[i];
    for (int i = tid; i <= N; i += MT) laboff_s[i] = a.lab_off[i];
    if (tid == 0) epoch_s = lb_epoch(a.ctl);
    __syncthreads();
    const unsigned epoch = epoch_s;
    const int q0 = a.q0;
    const int dsh = (int)(reinterpret_cast<uintptr_t>(a.x) & 15);
    const uint8_t *xa = a.x - dsh;
    const int64_t nP = a.n + dsh;
    int16_t *nxt = next_s[wv];
    long long *kc = kc_s[wv];
    uint8_t *stage = stage_s[wv];
    int32_t *own = own_s[wv];
    int32_t *tailw = tail_s[wv];
    int32_t *sizew = size_s[wv];
    long long T = 0, X = 0, M = 0;

    for (;;) {
        int sg = 0;
        if (lane == 0) sg = take_ticket(a.ctl);
        sg = __shfl(sg, 0);
        if (sg >= a.n_segs) break;
        const int64_t lo = (int64_t)sg * SEG;
        const int64_t hi = lo + SEG < a.n ? lo + SEG : a.n;
        long long base = 0;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 0)
                for (int g = lane; g < SEG; g += 64) kc[g] = 0;
            // the lane's entry: state (-1: none), tag list, instance count
            int st = -1, head = -1, tail = -1, sz = 0;
            bool any = false;
            int64_t wb = -1;  // staged window (shifted positions)
            for (int64_t p = lo; p < a.n && (p < hi || any); ++p) {
                const int64_t ps = p + dsh;
                if (ps >= wb + WIN || wb < 0) {
                    wb = ps & ~(int64_t)(WIN - 1);
                    const int64_t g0 = wb + 16 * lane;
                    const uint4 v = g0 < nP ? load_granule(xa, g0) : make_uint4(0, 0, 0, 0);
                    __builtin_amdgcn_wave_barrier();
                    *reinterpret_cast<uint4 *>(stage + 16 * lane) = v;
                    __builtin_amdgcn_wave_barrier();
                }
                const int b = stage[ps - wb];
                // step every entry (one lookup per entry, whatever it holds)
                int t = -1;
                if (st >= 0) {
                    const int v = tab_s[st * 256 + b];
                    t = v != 255 && (flags_s[v] & kLive) ? v : -1;
                    if (pass == 0) {
                        T += sz;
                        X += t >= 0 ? sz : 0;
                    }
                }
                // the instance started here, in the first free lane
                const unsigned long long used = __ballot(st >= 0);
                if (p < hi) {
                    const int f = __ffsll((long long)~used) - 1;
                    if (lane == f) {
                        const int g = (int)(p - lo);
                        const int v = tab_s[q0 * 256 + b];
                        t = v != 255 && (flags_s[v] & kLive) ? v : -1;
                        head = tail = g;
                        sz = 1;
                        nxt[g] = -1;
                        if (pass == 0) {
                            ++T;
                            X += t >= 0 ? 1 : 0;
                        }
                    }
                }
                // entries whose targets coincide merge into one lane
                if (t >= 0) own[t] = lane;
                __builtin_amdgcn_wave_barrier();
                const bool win = t >= 0 && own[t] == lane;
                const bool lose = t >= 0 && !win;
                if (__any(lose)) {
                    if (win) {
                        tailw[t] = tail;
                        sizew[t] = sz;
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (lose) {
                        const int old = atomicExch(&tailw[t], tail);
                        nxt[old] = (int16_t)head;
                        atomicAdd(&sizew[t], sz);
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (win) {
                        tail = tailw[t];
                        sz = sizew[t];
                    }
                }
                st = win ? t : -1;
                // report: every tag of an entry in a final state
                const bool fin = st >= 0 && (flags_s[st] & kFinal);
                if (__any(fin)) {
                    if (fin) {
                        const int l0 = laboff_s[st], l1 = laboff_s[st + 1];
                        const int L = l1 - l0;
                        if (pass == 0) {
                            M += (long long)L * sz;
                            for (int g = head; g >= 0; g = nxt[g]) kc[g] += L;
                        } else {
                            for (int g = head; g >= 0; g = nxt[g]) {
                                const long long k = kc[g];
                                for (int l = 0; l < L; ++l) {
                                    const long long at = base + k + l;
                                    if (at < a.cap) {
                                        MatchOut *o = &a.out[at];
                                        o->start = (int32_t)(lo + g);
                                        o->end = (int32_t)p;
                                        o->label = a.lab[l0 + l];
                                    }
                                }
                                kc[g] = k + L;
                            }
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                any = __any(st >= 0);
            }
            if (pass == 0) {
                // per-tag offsets within the segment, then the segment's base
                __builtin_amdgcn_wave_barrier();
                constexpr int PER = SEG / 64;
                long long own_sum = 0;
                for (int j = 0; j < PER; ++j) own_sum += kc[lane * PER + j];
                const long long inc = wave_incl_scan(own_sum);
                const long long seg_total = __shfl(inc, 63);
                long long run = inc - own_sum;
                for (int j = 0; j < PER; ++j) {
                    const long long c = kc[lane * PER + j];
                    kc[lane * PER + j] = run;
                    run += c;
                }
                __builtin_amdgcn_wave_barrier();
                const long long ex = lookback(a.lb, sg, epoch, seg_total);
                base = ex;
                if (sg == a.n_segs - 1 && lane == 0) *a.total = ex + seg_total;
                if (seg_total == 0) break;
            }
        }
    }
    long long st4[4] = {T, X, 0, M};
    block_sum4<MT>(st4, red4);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.bstats[4 * blockIdx.x + k] = st4[k];
    }
    finish_launch<MT>(a.ctl, a.lb, a.lb_cap, &last_s);
}

}  // namespace

hipError_t launch_dfa_merged(const MergedArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(dfa_merged_kernel, dim3(grid), dim3(MT), 0, s, a);
    return hipGetLastError();
}

const void *dfa_merged_fn() { return reinterpret_cast<const void *>(&dfa_merged_kernel); }

}  // namespace pfsmk
