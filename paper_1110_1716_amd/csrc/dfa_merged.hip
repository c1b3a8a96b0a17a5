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
//     the entry holds;
//   * entries whose targets coincide merge: one lane wins the target in an
//     LDS table, the others append their tag lists to its list through an
//     atomic exchange of the list tail (tag lists are linked through an LDS
//     array indexed by tag);
//   * the instance started at the current byte (while inside the segment)
//     joins the entry already in its state, else takes a free lane;
//   * an entry in a final state reports every label for every tag it holds.
// A scan is three launches: a count launch walks every segment once and
// stores each start's number of matches and the segment's total; one
// workgroup scans the segment totals; a write launch walks every segment
// again, turns its starts' counts into output offsets and stores the
// matches, so each start's matches come out in (end, label) order and starts
// in increasing order.  (A look-back between the two walks would make a
// wave wait for every earlier segment's count walk, whose lengths vary with
// the input.)
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
    // tab_s: the table by byte in dynamic LDS (n_states * 256 bytes): the
    // live target (bits 0-5) with bit 7 set when it is final, 255 = none
    extern __shared__ __align__(16) uint8_t tab_s[];
    __shared__ int32_t laboff_s[kMergedStates + 1];
    __shared__ int16_t next_s[MW][SEG];   // tag list links (-1: end)
    // matches per tag, then output offsets, in 32 bits up to a.narrow_max;
    // counts that would pass it continue in 64 bits in a.tag_cnt (spill_s
    // marks those tags), and a segment whose total passes it keeps its
    // offsets there
    __shared__ int32_t kc_s[MW][SEG];
    __shared__ unsigned long long spill_s[MW][SEG / 64];
    __shared__ uint8_t stage_s[MW][WIN];
    __shared__ int32_t own_s[MW][64], tail_s[MW][64], size_s[MW][64];
    __shared__ long long red4[4 * MW];
    __shared__ int last_s;

    const int tid = threadIdx.x;
    const int wv = tid >> 6;
    const int lane = lane_id();
    const int N = a.n_states;
    for (int i = tid; i < N * 256; i += MT) tab_s[i] = a.tab[i];
    for (int i = tid; i <= N; i += MT) laboff_s[i] = a.lab_off[i];
    __syncthreads();
    const int q0 = a.q0;
    const int dsh = (int)(reinterpret_cast<uintptr_t>(a.x) & 15);
    const uint8_t *xa = a.x - dsh;
    const int64_t nP = a.n + dsh;
    int16_t *nxt = next_s[wv];
    int32_t *kc = kc_s[wv];
    unsigned long long *spill = spill_s[wv];
    const int lim = a.narrow_max;
    uint8_t *stage = stage_s[wv];
    int32_t *own = own_s[wv];
    int32_t *tailw = tail_s[wv];
    int32_t *sizew = size_s[wv];
    long long T = 0, X = 0, M = 0;
    // the lane's 16 bytes of the staged window at wb (shifted positions)
    auto fetch = [&](int64_t wb) __attribute__((always_inline)) {
        const int64_t g0 = wb + 16 * lane;
        return g0 >= 0 && g0 < nP ? load_granule(xa, g0) : make_uint4(0, 0, 0, 0);
    };

    for (;;) {
        int sg = 0;
        if (lane == 0) sg = take_ticket(a.ctl);
        sg = __shfl(sg, 0);
        if (sg >= a.n_segs) break;
        const int64_t lo = (int64_t)sg * SEG;
        const int64_t hi = lo + SEG < a.n ? lo + SEG : a.n;
        const int pass = a.pass;
        long long base = 0;
        bool wide = false;  // offsets kept in a.tag_cnt (64 bits)
        if (pass == 0) {
            for (int g = lane; g < SEG; g += 64) kc[g] = 0;
            if (lane < SEG / 64) spill[lane] = 0;
        } else {
            // this segment's starts: output offsets from their counts
            base = a.seg_base[sg];
            if (a.seg_base[sg + 1] == base) continue;  // no matches
            wide = a.seg_base[sg + 1] - base > lim;
            constexpr int PER = SEG / 64;
            long long own_sum = 0;
            for (int j = 0; j < PER; ++j) {
                const int64_t i = lo + lane * PER + j;
                own_sum += i < hi ? a.tag_cnt[i] : 0;
            }
            const long long inc = wave_incl_scan(own_sum);
            long long run = inc - own_sum;
            for (int j = 0; j < PER; ++j) {
                const int64_t i = lo + lane * PER + j;
                const long long c = i < hi ? a.tag_cnt[i] : 0;
                if (!wide) kc[lane * PER + j] = (int32_t)run;
                else if (i < hi) a.tag_cnt[i] = run;
                run += c;
            }
            if (wide) __threadfence();  // the offsets reach L2 before the atomics below
            __builtin_amdgcn_wave_barrier();
        }
        {
            // the lane's entry: state (-1: none) and whether it is final, its
            // tag list and instance count
            int st = -1, head = -1, tail = -1, sz = 0;
            bool stf = false, any = false;
            // stage the first window, request the next; bn: the next byte
            int64_t wb = (lo + dsh) & ~(int64_t)(WIN - 1);
            const uint4 first = fetch(wb);
            uint4 pre = fetch(wb + WIN);
            __builtin_amdgcn_wave_barrier();
            *reinterpret_cast<uint4 *>(stage + 16 * lane) = first;
            __builtin_amdgcn_wave_barrier();
            int bn = stage[lo + dsh - wb];
            for (int64_t p = lo; p < a.n && (p < hi || any); ++p) {
                const int b = bn;
                const int64_t ps1 = p + 1 + dsh;
                if (ps1 >= wb + WIN) {
                    wb += WIN;
                    __builtin_amdgcn_wave_barrier();
                    *reinterpret_cast<uint4 *>(stage + 16 * lane) = pre;
                    __builtin_amdgcn_wave_barrier();
                    pre = fetch(wb + WIN);
                }
                bn = stage[ps1 - wb];
                // step every entry (one lookup per entry, whatever it holds)
                // and find the state of the instance started here
                int t = -1, t0 = -1;
                bool tf = false, t0f = false;
                if (st >= 0) {
                    const int v = tab_s[st * 256 + b];
                    t = v == 255 ? -1 : (v & 63);
                    tf = v != 255 && (v & 128);
                }
                if (p < hi) {
                    const int v = tab_s[q0 * 256 + b];
                    t0 = v == 255 ? -1 : (v & 63);
                    t0f = v != 255 && (v & 128);
                }
                if (pass == 0) {
                    T += sz;
                    X += t >= 0 ? sz : 0;
                    if (p < hi && lane == 0) {
                        ++T;
                        X += t0 >= 0 ? 1 : 0;
                    }
                }
                // entries whose targets coincide merge into one lane (only
                // possible with two or more survivors)
                const unsigned long long alive = __ballot(t >= 0);
                bool win = t >= 0;
                if (__popcll(alive) >= 2) {
                    if (t >= 0) own[t] = lane;
                    __builtin_amdgcn_wave_barrier();
                    win = t >= 0 && own[t] == lane;
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
                }
                st = win ? t : -1;
                stf = win && tf;
                if (!win) sz = 0;
                // the new instance joins the entry in its state, or takes a
                // free lane (entries hold distinct states, at most 63)
                if (t0 >= 0) {
                    const int g = (int)(p - lo);
                    const unsigned long long hit = __ballot(st == t0);
                    const int w = hit ? __ffsll((long long)hit) - 1 : __ffsll((long long)~__ballot(st >= 0)) - 1;
                    if (lane == w) {
                        nxt[g] = -1;
                        if (hit) {
                            nxt[tail] = (int16_t)g;
                            tail = g;
                            ++sz;
                        } else {
                            st = t0;
                            stf = t0f;
                            head = tail = g;
                            sz = 1;
                        }
                    }
                }
                // report: every tag of an entry in a final state
                const bool fin = st >= 0 && stf;
                if (__any(fin)) {
                    if (fin) {
                        const int l0 = laboff_s[st], l1 = laboff_s[st + 1];
                        const int L = l1 - l0;
                        if (pass == 0) {
                            M += (long long)L * sz;
                            for (int g = head; g >= 0; g = nxt[g]) {
                                const int k = kc[g];
                                if (k > lim - L) {
                                    // the count leaves 32 bits: move it to memory
                                    unsigned long long *slot =
                                        reinterpret_cast<unsigned long long *>(&a.tag_cnt[lo + g]);
                                    const unsigned long long add = (unsigned long long)((long long)k + L);
                                    const unsigned long long bit = 1ull << (g & 63);
                                    if (spill[g >> 6] & bit) {
                                        atomicAdd(slot, add);
                                    } else {
                                        atomicExch(slot, add);
                                        spill[g >> 6] |= bit;
                                    }
                                    kc[g] = 0;
                                } else {
                                    kc[g] = k + L;
                                }
                            }
                        } else {
                            // (the first label is read once: the output
                            // stores would otherwise force a reload per tag)
                            const int32_t lab0 = L > 0 ? a.lab[l0] : 0;
                            for (int g = head; g >= 0; g = nxt[g]) {
                                long long k;
                                if (wide) {
                                    k = (long long)atomicAdd(
                                        reinterpret_cast<unsigned long long *>(&a.tag_cnt[lo + g]),
                                        (unsigned long long)L);
                                } else {
                                    k = kc[g];
                                    kc[g] = (int32_t)(k + L);
                                }
                                for (int l = 0; l < L; ++l) {
                                    const long long at = base + k + l;
                                    if (at < a.cap) {
                                        MatchOut *o = &a.out[at];
                                        o->start = (int32_t)(lo + g);
                                        o->end = (int32_t)p;
                                        o->label = l == 0 ? lab0 : a.lab[l0 + l];
                                    }
                                }
                            }
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                any = __any(st >= 0);
            }
            if (pass == 0) {
                // each start's count, and the segment's total
                __builtin_amdgcn_wave_barrier();
                long long sum = 0;
                for (int g = lane; g < SEG; g += 64) {
                    const int64_t i = lo + g;
                    if (i < hi) {
                        long long c = kc[g];
                        if ((spill[g >> 6] >> (g & 63)) & 1)  // read back at L2
                            c += (long long)atomicAdd(reinterpret_cast<unsigned long long *>(&a.tag_cnt[i]), 0ull);
                        a.tag_cnt[i] = c;
                        sum += c;
                    }
                }
                sum = wave_sum(sum);
                if (lane == 0) a.seg_cnt[sg] = sum;
            }
        }
    }
    if (a.pass == 0) {
        long long st4[4] = {T, X, 0, M};
        block_sum4<MT>(st4, red4);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) a.bstats[4 * blockIdx.x + k] = st4[k];
        }
    }
    finish_launch<MT>(a.ctl, a.lb, a.lb_cap, &last_s);
}

// Exclusive scan of the segment totals (one workgroup): seg_base[s] for
// s <= n_segs, and the grand total.
__global__ __launch_bounds__(1024) void merged_seg_scan_kernel(const long long *seg_cnt, int n_segs,
                                                               long long *seg_base, int64_t *total) {
    __shared__ long long red[16];
    long long run = 0;
    for (int c0 = 0; c0 < n_segs; c0 += 1024) {
        const int s = c0 + threadIdx.x;
        long long tot;
        const long long ex = block_excl_scan<1024>(s < n_segs ? seg_cnt[s] : 0, red, &tot);
        if (s < n_segs) seg_base[s] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        seg_base[n_segs] = run;
        *total = run;
    }
}

}  // namespace

hipError_t launch_dfa_merged(const MergedArgs &a0, int grid, hipStream_t s) {
    MergedArgs a = a0;
    a.pass = 0;
    hipLaunchKernelGGL(dfa_merged_kernel, dim3(grid), dim3(MT), merged_lds(a.n_states), s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(merged_seg_scan_kernel, dim3(1), dim3(1024), 0, s, a.seg_cnt, a.n_segs, a.seg_base, a.total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    a.pass = 1;
    hipLaunchKernelGGL(dfa_merged_kernel, dim3(grid), dim3(MT), merged_lds(a.n_states), s, a);
    return hipGetLastError();
}

const void *dfa_merged_fn() { return reinterpret_cast<const void *>(&dfa_merged_kernel); }

}  // namespace pfsmk
