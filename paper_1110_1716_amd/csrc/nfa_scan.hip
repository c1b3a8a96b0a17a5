// All-matches NFA scan for gfx950 (Section III.B with epsilon transitions;
// the NFA case of Section III.C).
//
// Grid of 256-thread workgroups that take segments from a ticket counter; a
// workgroup owns the start positions of its segment (lazy data
// partitioning, Section III.D.2).  For each start i the instance's state set
// is advanced one symbol at a time (Section III.B steps 3-4), closed under
// epsilon edges right after each symbol, and every label of every final
// state in it is reported with end = the symbol's position.
//   * Symbols one and two come from read-only caches derived from the
//     automaton when it is loaded: the set after the first symbol for each
//     byte (the epsilon closure of q0 needs no work per position) and, for
//     each byte pair, the set after two symbols, located through a 64 Ki-bit
//     bitmap in LDS.  Most instances end there.
//   * Live instances keep their set in registers (up to kNfaK states, kept
//     duplicate-free, so every state is expanded once per symbol) and wait in
//     a wave-private LDS queue; each queue round advances every walk through
//     the rest of a 16-byte input chunk, one packed 32-byte state record load
//     per state and symbol.  A lane holds two walks, which step together so
//     that their record loads overlap.
//   * An instance whose set outgrows kNfaK is replayed by the whole workgroup
//     from its start: frontier lists and a visited bitset in global scratch,
//     the matches it had already reported skipped.
//   * Matches go to an LDS buffer keyed by (start - segment start, k), k the
//     instance's match count so far; labels of one symbol are reported in
//     increasing order, so k orders (end, label) within a start.  Offsets come
//     from decoupled look-back over the segment tickets as in the DFA scan; a
//     segment whose matches overflow the buffer is walked again 256 starts at
//     a time to count, scan and write.
#include "dfa_defer.h"
#include "scan_common.h"
#include "stream.h"

namespace pfsmk {

namespace {

constexpr int NT = kNfaThreads;
constexpr int W = kNfaWindow;
constexpr int K = kNfaK;  // states a queued walk keeps
constexpr int QW = kNfaQueue * 2;
constexpr int QK = QW / 64;
constexpr int MC = kNfaMatchCap;
constexpr int BC = kNfaBigCap;

struct Walk {
    int32_t start, pos, k, n;
    uint32_t s[K];
};

struct Big {
    int32_t start, k0, pos0, pad;
};

// A walk waiting for a gap pass: its set is n gap states marked kRecGapFin
// (each with at most 64 any-byte steps left, their chains distinct); next
// symbol at pos, k matches reported so far.
struct GapEnt {
    int32_t start, pos, k, n;
    uint32_t s[K];
};
constexpr int GC = kNfaGapCap;
constexpr int LC = 64 + 8 * 64;  // list: fewer than 64 left over plus one half-window of starts
// A round adds at most QW walks to fewer than 64 waiting; during a pass at
// most QW - 1 wait, so the last 64 entries hold a 32-byte bitmap per lane.
static_assert(sizeof(GapEnt) >= 32 && GC >= 64 + QW, "gap list too small");

// Where a walk's matches go.
enum Mode : int { kBuffer = 0, kCount = 1, kWrite = 2 };

// kCarry: instances live at the end of the input are collected (streams);
// plain scans compile those paths out.
template <bool kCarry>
struct NfaCtx {
    static constexpr bool kCarryOn = kCarry;
    const NfaArgs &a;
    const uint32_t *pbits_s;
    const int32_t *f1o_s;
    const int32_t *e1o_s;
    uint32_t *mkey;
    int32_t *mend;
    int32_t *mlab;
    int *mn;
    int *ovf;
    int64_t seg_lo = 0;   // the segment's first start (shifted position)
    int32_t n32 = 0;      // end of the stream (shifted position)
    // Positions are shifted by dsh, the stream's offset from the 16-byte
    // boundary below it: position p is byte p of the aligned base xa, and
    // reported positions are p - dsh.
    const uint8_t *xa = nullptr;
    int64_t nP = 0;
    int32_t dsh = 0;
    long long T = 0, X = 0, L = 0, M = 0;

    // Record one match of the instance started at `start`.  k is the number
    // of matches it reported before this one.
    __device__ __forceinline__ void put(int mode, int32_t start, int32_t end, int32_t label, int32_t k,
                                        long long at) {
        if (mode == kBuffer) {
            ++M;
            if (*ovf) return;
            const int slot = atomicAdd(mn, 1);
            if (slot < MC) {
                mkey[slot] = ((uint32_t)(start - seg_lo) << 16) | (uint32_t)(k & 0xffff);
                mend[slot] = end - dsh;
                mlab[slot] = label;
            } else {
                *ovf = 1;
            }
        } else if (mode == kWrite) {
            if (at + k < a.cap) {
                MatchOut *p = &a.out[at + k];
                p->start = start - dsh;
                p->end = end - dsh;
                p->label = label;
            }
        }
    }
    // The instance started at `start` holds the n states of S after the last
    // byte of the input: hand it to the next piece when carries are
    // collected.
    __device__ __forceinline__ void carry_set(int32_t start, const uint32_t (&S)[K], int n) const {
        if constexpr (!kCarry) return;
        const unsigned long long slot = carry_reserve(a.carry, n);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < n) carry_write(a.carry, slot + j, start - dsh, S[j] & kStateMask);
    }
    // The same for the set after the first symbol c1 (start = the last byte).
    __device__ __forceinline__ void carry_first(int32_t start, int c1) const {
        if constexpr (!kCarry) return;
        const int lo = f1o_s[c1], hi = f1o_s[c1 + 1];
        const unsigned long long slot = carry_reserve(a.carry, hi - lo);
        for (int j = lo; j < hi; ++j) carry_write(a.carry, slot + (j - lo), start - dsh, a.f1[j] & kStateMask);
    }
};

__device__ __forceinline__ bool edge_matches(const NfaArgs &a, uint32_t test, int byte) {
    const uint32_t kind = (test >> 8) & 3u;
    if (kind == 0) return (int)(test & 255u) == byte;
    if (kind == 1) return true;
    return (a.class_bits[(size_t)(test >> 10) * 8 + (byte >> 5)] >> (byte & 31)) & 1u;
}

// Duplicate-free insertion of a target word into O[0..nO); false when the
// set would exceed K.
__device__ __forceinline__ bool set_insert(uint32_t (&O)[K], int &nO, uint32_t w) {
    const uint32_t q = w & kStateMask;
    bool dup = false;
#pragma unroll
    for (int j = 0; j < K; ++j) dup |= (j < nO) && ((O[j] & kStateMask) == q);
    if (dup) return true;
    if (nO >= K) return false;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j == nO) O[j] = w;
    ++nO;
    return true;
}

__device__ __forceinline__ bool add_target(const NfaArgs &a, uint32_t (&O)[K], int &nO, uint32_t tgt) {
    if (!(tgt & kTgtList)) return set_insert(O, nO, tgt);
    const int idx = (int)(tgt & ~kTgtList);
    bool ok = true;
    for (int j = a.cl_off[idx]; j < a.cl_off[idx + 1] && ok; ++j) ok = set_insert(O, nO, a.cl[j]);
    return ok;
}

// One symbol for a set whose state records are already loaded:
// O = closure(delta(S, byte)) over live states.  Returns false when O would
// exceed K states.
__device__ __forceinline__ bool nfa_step_rec(const NfaArgs &a, const NfaRec (&r)[K], int nS, int byte,
                                             uint32_t (&O)[K], int &nO) {
    nO = 0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < nS && ok) {
            if (r[j].info & kRecInline) {
                if (r[j].n_edges > 0 && edge_matches(a, r[j].e0_test, byte)) ok = add_target(a, O, nO, r[j].e0_tgt);
                if (ok && r[j].n_edges > 1 && edge_matches(a, r[j].e1_test, byte))
                    ok = add_target(a, O, nO, r[j].e1_tgt);
            } else {
                for (int e = 0; e < r[j].n_edges && ok; ++e) {
                    const uint2 ed = reinterpret_cast<const uint2 *>(a.edges)[r[j].edge_off + e];
                    if (edge_matches(a, ed.x, byte)) ok = add_target(a, O, nO, ed.y);
                }
            }
        }
    }
    return ok;
}

// One symbol for a set: O = closure(delta(S, byte)) over live states.
// Returns false when O would exceed K states.
__device__ __forceinline__ bool nfa_step(const NfaArgs &a, const uint32_t (&S)[K], int nS, int byte,
                                         uint32_t (&O)[K], int &nO) {
    NfaRec r[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < nS) r[j] = a.rec[S[j] & kStateMask];
    return nfa_step_rec(a, r, nS, byte, O, nO);
}

// Report the labels of the final states of O (ascending, once each).
template <class Ctx>
__device__ __forceinline__ void emit_set(Ctx &c, int mode, const uint32_t (&O)[K], int nO, int32_t start,
                                         int32_t end, int32_t &k, int32_t k0, long long at) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) any |= (j < nO) && (O[j] & kTgtFinal);
    if (!any) return;
    int lo[K], hi[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        lo[j] = hi[j] = 0;
        if (j < nO && (O[j] & kTgtFinal)) {
            const NfaRec &r = c.a.rec[O[j] & kStateMask];
            lo[j] = r.lab_off;
            hi[j] = r.lab_off + (int)(r.info >> 8);
        }
    }
    int last = -1;
    for (;;) {
        int m = 0x7fffffff;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            while (lo[j] < hi[j] && c.a.lab[lo[j]] <= last) ++lo[j];
            if (lo[j] < hi[j]) m = min(m, c.a.lab[lo[j]]);
        }
        if (m == 0x7fffffff) break;
        if (k >= k0) c.put(mode, start, end, m, k, at);
        ++k;
        last = m;
    }
}

// Report a sorted unique label list.
template <class Ctx>
__device__ __forceinline__ void emit_list(Ctx &c, int mode, const int32_t *lab, int lo, int hi, int32_t start,
                                          int32_t end, int32_t &k, int32_t k0, long long at) {
    for (int l = lo; l < hi; ++l, ++k)
        if (k >= k0) c.put(mode, start, end, lab[l], k, at);
}

// Sets after the first two symbols of start i (when i + 1 < n).  Returns the
// number of states in the second set, or -1 when it exceeds K (S untouched).
template <class Ctx>
__device__ __forceinline__ int first_two(Ctx &c, int c1, int c2, uint32_t (&S)[K], int &pair_lab_lo,
                                         int &pair_lab_hi, bool &overflow) {
    const NfaArgs &a = c.a;
    overflow = false;
    pair_lab_lo = pair_lab_hi = 0;
    int nS = 0;
    if (a.pair_on) {
        const int p = c1 * 256 + c2;
        if (!((c.pbits_s[p >> 5] >> (p & 31)) & 1u)) return 0;
        const PairRange r = a.p_rng[p];
        const int s_lo = r.st_lo, s_hi = r.st_hi;
        pair_lab_lo = r.lab_lo;
        pair_lab_hi = r.lab_hi;
        const int cnt = s_hi - s_lo;
        if (cnt > K) {
            overflow = true;
            return cnt;
        }
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < cnt) S[j] = a.p_st[s_lo + j];
        return cnt;
    }
    // No pair cache: expand the first-symbol set directly.
    for (int j = c.f1o_s[c1]; j < c.f1o_s[c1 + 1]; ++j) {
        const NfaRec r = a.rec[a.f1[j] & kStateMask];
        bool ok = true;
        if (r.info & kRecInline) {
            if (r.n_edges > 0 && edge_matches(a, r.e0_test, c2)) ok = add_target(a, S, nS, r.e0_tgt);
            if (ok && r.n_edges > 1 && edge_matches(a, r.e1_test, c2)) ok = add_target(a, S, nS, r.e1_tgt);
        } else {
            for (int e = 0; e < r.n_edges && ok; ++e) {
                const uint2 ed = reinterpret_cast<const uint2 *>(a.edges)[r.edge_off + e];
                if (edge_matches(a, ed.x, c2)) ok = add_target(a, S, nS, ed.y);
            }
        }
        if (!ok) {
            overflow = true;
            return K + 1;
        }
    }
    return nS;
}

// The labels reported after the second symbol when there is no pair cache
// (finals among S); with the cache they come from the pair's label list.
//
// Full walk of one start by one lane, for the count and write passes of a
// dense segment.  Returns the number of matches, or -1 when a set outgrows K
// (the caller replays that start with the whole workgroup).  With `work`,
// its instance-steps and state activations are added to c.T and c.X (only
// when the walk completes).
template <class Ctx>
__device__ __forceinline__ long long walk_lane(Ctx &c, int32_t i, int mode, long long at, bool work = false) {
    const NfaArgs &a = c.a;
    int32_t k = 0;
    const int c1 = c.xa[i];
    const int n1 = c.f1o_s[c1 + 1] - c.f1o_s[c1];
    long long nT = 1, nX = n1;
    if (n1 == 0) {
        if (work) ++c.T;
        return 0;
    }
    emit_list(c, mode, a.e1, c.e1o_s[c1], c.e1o_s[c1 + 1], i, i, k, 0, at);
    if (i + 1 >= c.n32) {
        if (mode == kCount) c.carry_first(i, c1);
        if (work) {
            c.T += nT;
            c.X += nX;
        }
        return k;
    }
    uint32_t S[K];
    int llo, lhi;
    bool ovf;
    int nS = first_two(c, c1, c.xa[i + 1], S, llo, lhi, ovf);
    if (ovf) return -1;
    if (a.pair_on) emit_list(c, mode, a.p_lab, llo, lhi, i, i + 1, k, 0, at);
    else emit_set(c, mode, S, nS, i, i + 1, k, 0, at);
    ++nT;
    nX += nS;
    int32_t pos = i + 2;
    while (nS > 0 && pos < c.n32) {
        uint32_t O[K];
        int nO;
        if (!nfa_step(a, S, nS, c.xa[pos], O, nO)) return -1;
        ++nT;
        nX += nO;
        emit_set(c, mode, O, nO, i, pos, k, 0, at);
#pragma unroll
        for (int j = 0; j < K; ++j) S[j] = O[j];
        nS = nO;
        ++pos;
    }
    if (nS > 0 && mode == kCount) c.carry_set(i, S, nS);
    if (work) {
        c.T += nT;
        c.X += nX;
    }
    return k;
}

__device__ __forceinline__ int block_min(int v, int *redi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    if (lane_id() == 0) redi[threadIdx.x >> 6] = v;
    __syncthreads();
    int m = redi[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) m = min(m, redi[i]);
    __syncthreads();
    return m;
}

// One symbol for a frontier held by the whole workgroup: nxt receives
// closure(delta(cur, byte)) over live states, duplicate-free (bits marks the
// states taken and is clear again on return).  Returns the size of nxt on
// every thread.  Contains barriers; sh[0] must be 0 on entry and is again on
// return.
__device__ __forceinline__ int frontier_step(const NfaArgs &a, const uint32_t *cur, int nF, int byte, uint32_t *nxt,
                                             uint32_t *bits, int *sh) {
    const int tid = threadIdx.x;
    for (int j = tid; j < nF; j += NT) {
        const NfaRec r = a.rec[cur[j] & kStateMask];
        const int ne = r.n_edges;
        for (int e = 0; e < ne; ++e) {
            uint32_t test, tgt;
            if (r.info & kRecInline) {
                test = e == 0 ? r.e0_test : r.e1_test;
                tgt = e == 0 ? r.e0_tgt : r.e1_tgt;
            } else {
                const uint2 ed = reinterpret_cast<const uint2 *>(a.edges)[r.edge_off + e];
                test = ed.x;
                tgt = ed.y;
            }
            if (!edge_matches(a, test, byte)) continue;
            int lo = 0, hi = 1;
            if (tgt & kTgtList) {
                const int idx = (int)(tgt & ~kTgtList);
                lo = a.cl_off[idx];
                hi = a.cl_off[idx + 1];
            }
            for (int t = lo; t < hi; ++t) {
                const uint32_t w = (tgt & kTgtList) ? a.cl[t] : tgt;
                const uint32_t q = w & kStateMask;
                const uint32_t bit = 1u << (q & 31);
                const uint32_t old = atomicOr(&bits[q >> 5], bit);
                if (!(old & bit)) nxt[atomicAdd(&sh[0], 1)] = w;
            }
        }
    }
    __syncthreads();
    const int nN = sh[0];
    __syncthreads();
    for (int j = tid; j < nN; j += NT) {
        const uint32_t q = nxt[j] & kStateMask;
        atomicAnd(&bits[q >> 5], ~(1u << (q & 31)));
    }
    if (tid == 0) sh[0] = 0;
    return nN;
}

// The labels of the final states of a frontier, ascending and once each:
// emit(label) runs on every thread for each, in that order.  Contains
// barriers (sh[1 .. NT/64] are used).
template <class F>
__device__ __forceinline__ void frontier_labels(const NfaArgs &a, const uint32_t *front, int nN, int *sh, F &&emit) {
    const int tid = threadIdx.x;
    int last = -1;
    for (;;) {
        int mine = 0x7fffffff;
        for (int j = tid; j < nN; j += NT) {
            if (!(front[j] & kTgtFinal)) continue;
            const NfaRec r = a.rec[front[j] & kStateMask];
            const int hi = r.lab_off + (int)(r.info >> 8);
            for (int l = r.lab_off; l < hi; ++l) {
                const int v = a.lab[l];
                if (v > last) {
                    mine = min(mine, v);
                    break;
                }
            }
        }
        const int m = block_min(mine, sh + 1);
        if (m == 0x7fffffff) break;
        emit(m);
        last = m;
    }
}

// Replay of start s by the whole workgroup with unbounded sets (frontiers in
// global scratch).  Matches before the k0-th are skipped (already reported);
// work counters are kept for positions >= pos0 (earlier ones were counted).
// Returns the number of matches reported from k0 on (every thread).
template <class Ctx>
__device__ __forceinline__ long long walk_block(Ctx &c, int32_t s, int32_t k0, int32_t pos0, int mode, long long at,
                                uint32_t *F0, uint32_t *F1, uint32_t *bits, int *sh) {
    // sh[0]: next frontier size, sh[1..NT/64]: reduction slots
    const NfaArgs &a = c.a;
    const int tid = threadIdx.x;
    const int c1 = c.xa[s];
    int nF = c.f1o_s[c1 + 1] - c.f1o_s[c1];
    for (int j = tid; j < nF; j += NT) F0[j] = a.f1[c.f1o_s[c1] + j];
    int32_t k = 0;  // tracked by every thread identically
    if (tid == 0) {
        if (s >= pos0) {
            ++c.T;
            c.X += nF;
        }
        emit_list(c, mode, a.e1, c.e1o_s[c1], c.e1o_s[c1 + 1], s, s, k, k0, at);
    } else {
        k += c.e1o_s[c1 + 1] - c.e1o_s[c1];
    }
    if (tid == 0) sh[0] = 0;
    __syncthreads();
    uint32_t *cur = F0, *nxt = F1;
    int32_t pos = s + 1;
    while (nF > 0 && pos < c.n32) {
        const int nN = frontier_step(a, cur, nF, c.xa[pos], nxt, bits, sh);
        if (tid == 0 && pos >= pos0) {
            ++c.T;
            c.X += nN;
        }
        frontier_labels(a, nxt, nN, sh, [&](int m) {
            if (tid == 0 && k >= k0) c.put(mode, s, pos, m, k, at);
            ++k;
        });
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
        nF = nN;
        ++pos;
        __syncthreads();
    }
    if (Ctx::kCarryOn && nF > 0 && mode != kWrite)
        for (int j = tid; j < nF; j += NT)
            carry_write(a.carry, carry_reserve(a.carry, 1), s - c.dsh, cur[j] & kStateMask);
    __syncthreads();
    return (long long)k - k0;
}

// One queue round of this wave: every walk advances through the rest of the
// 16-byte chunk holding its next position.  Walks whose set outgrows K go to
// the workgroup's replay list.  A lane's walks advance together, one symbol
// each per step, and the state records of all of them are requested before
// any is used, so their L2 round trips overlap.
// Which of 16 bytes an edge test accepts (bit k for byte k of v).  A
// single byte is compared four at a time (a byte of w ^ the repeated byte is
// zero exactly when 0x80 ends up set in it); a class reads its bitmap from
// bm, a 32-byte copy in LDS.
__device__ __forceinline__ uint32_t test16(uint32_t test, const uint8_t *bm, uint4 v) {
    const uint32_t kind = (test >> 8) & 3u;
    if (kind == 1) return 0xffffu;
    uint32_t r = 0;
    if (kind == 0) {
        const uint32_t rep = (test & 255u) * 0x01010101u;
        const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w = q[i] ^ rep;
            const uint32_t z = ~(((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w | 0x7f7f7f7fu);
            r |= (((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u)) << (4 * i);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int b = byte_of(v, k);
            r |= ((uint32_t)(bm[b >> 3] >> (b & 7)) & 1u) << k;
        }
    }
    return r;
}

// The bytes [base, base + 96) that an edge test accepts, as a 96-bit mask
// (h0: offsets 0-63, h1: 64-95).  A class bitmap is first copied to bm.
template <class Ctx>
__device__ __forceinline__ void mask96(Ctx &c, uint32_t test, uint8_t *bm, int32_t base, unsigned long long &h0,
                                       unsigned long long &h1) {
    if (((test >> 8) & 3u) == 2) {
        const uint4 *p = reinterpret_cast<const uint4 *>(c.a.class_bits + (size_t)(test >> 10) * 8);
        const uint4 b0 = p[0], b1 = p[1];
        reinterpret_cast<uint4 *>(bm)[0] = b0;
        reinterpret_cast<uint4 *>(bm)[1] = b1;
    }
    uint4 G0, G1, G2, G3, G4, G5;
    {
        const uint4 z = make_uint4(0, 0, 0, 0);
        G0 = base < c.nP ? load_granule(c.xa, base) : z;
        G1 = base + 16 < c.nP ? load_granule(c.xa, base + 16) : z;
        G2 = base + 32 < c.nP ? load_granule(c.xa, base + 32) : z;
        G3 = base + 48 < c.nP ? load_granule(c.xa, base + 48) : z;
        G4 = base + 64 < c.nP ? load_granule(c.xa, base + 64) : z;
        G5 = base + 80 < c.nP ? load_granule(c.xa, base + 80) : z;
        c.L += 6;
    }
    h0 = 0;
    h1 = 0;
    // The granules move down one register per chunk.
#pragma unroll 1
    for (int t = 0; t < 6; ++t) {
        const uint4 v = G0;
        G0 = G1;
        G1 = G2;
        G2 = G3;
        G3 = G4;
        G4 = G5;
        const unsigned long long m = test16(test, bm, v);
        if (t < 4) h0 |= m << (16 * t);
        else h1 |= m << (16 * (t - 4));
    }
}

// Bits [lo, hi] of a 128-bit mask (h0: bits 0-63, h1: 64-127); empty when
// hi < lo.
__device__ __forceinline__ void range_bits(int lo, int hi, unsigned long long &h0, unsigned long long &h1) {
    auto upto = [](int x) -> unsigned long long {  // bits [0, x) of a 64-bit word, x in [0, 64]
        return x <= 0 ? 0ull : (x >= 64 ? ~0ull : (1ull << x) - 1ull);
    };
    h0 = upto(hi + 1) & ~upto(lo);
    h1 = upto(hi + 1 - 64) & ~upto(lo - 64);
}

// Report the labels of final state w (a target word) at `end`.
template <class Ctx>
__device__ __forceinline__ void emit_state(Ctx &c, uint32_t w, int32_t start, int32_t end, int32_t &k) {
    const NfaRec r = c.a.rec[w & kStateMask];
    const int hi = r.lab_off + (int)(r.info >> 8);
    int last = -1;
    for (int l = r.lab_off; l < hi; ++l) {
        const int lab = c.a.lab[l];
        if (lab <= last) continue;
        c.put(kBuffer, start, end, lab, k, 0);
        ++k;
        last = lab;
    }
}

// Gap pass: up to 64 waiting gap walks, one per lane, each finished at once.
// From a gap state g with r any-byte steps left at position pos, the
// instance holds the next gap state after each of the symbols pos .. pos +
// r - 1, and each symbol p in [pos, pos + r] that E accepts starts an
// attempt along the chain after E.  Attempts started at different symbols
// are at different chain states at any time, and the chains of different
// gaps never meet, so the set sizes add up: X gains the gap states plus
// every attempt's length, the instance lives until the latest of them ends
// (T counts up to the symbol after it), and attempts that reach a chain's
// final end report, in order of their first symbol (which is also the order
// of their ends).  The bytes of [pos, pos + 80] come from six 16-byte loads
// issued together; E is tested on all of them, the chain's first edge too
// when E accepts some, and only attempts that pass both read on.  Reports of two or more gaps
// would interleave: such a walk is replayed by the workgroup instead.
template <class Ctx>
__device__ __forceinline__ void gap_pass(Ctx &c, GapEnt *gl, int &gcount, Big *big_s, int *nbig) {
    const NfaArgs &a = c.a;
    const int lane = lane_id();
    const int take = gcount < 64 ? gcount : 64;
    const bool act = lane < take;
    GapEnt g;
    g.n = 0;
    if (act) g = gl[lane];
    __builtin_amdgcn_wave_barrier();
    for (int e = 64 + lane; e < gcount; e += 64) gl[e - 64] = gl[e];
    __builtin_amdgcn_wave_barrier();
    gcount -= take;
    if (!act) return;
    const int32_t n = c.n32, pos = g.pos;
    const int32_t base = pos & ~15;
    // The list's last 64 entries are free during a pass (fewer than 128
    // wait): one 32-byte slot per lane holds a class bitmap.
    uint8_t *bm = reinterpret_cast<uint8_t *>(gl + GC - 64 + lane);
    // One iteration per gap state, then one more that reports for the only
    // gap whose attempts reach their chain's end (if there is one).
    uint32_t q0 = g.s[0], q1 = g.s[1], q2 = g.s[2], q3 = g.s[3], qm = 0;
    int nm = 0;
    long long X = 0;
    int32_t last = pos - 1;
    int32_t k = g.k;
#pragma unroll 1
    for (int it = 0; it <= g.n; ++it) {
        const bool em = it == g.n;
        uint32_t w;
        if (em) {
            if (nm != 1) break;
            w = qm;
        } else {
            w = q0;
            q0 = q1;
            q1 = q2;
            q2 = q3;
        }
        const NfaRec gr = a.rec[w & kStateMask];
        const int32_t rr = gr.edge_off;  // any-byte steps left, at least 1
        const uint32_t u0 = gr.e0_tgt;
        const bool end0 = (u0 & kTgtFinal) != 0;  // E's target ends the chain
        // hE: E accepts the byte at offset o from base.
        unsigned long long hE0, hE1;
        mask96(c, gr.e0_test, bm, base, hE0, hE1);
        // Attempts start at [pos, pe]; a second chain state needs one more byte.
        const int32_t pe = pos + rr < n - 1 ? pos + rr : n - 1;
        unsigned long long w0, w1, v0, v1;
        range_bits(pos - base, pe - base, w0, w1);
        range_bits(pos - base, (pe < n - 2 ? pe : n - 2) - base, v0, v1);
        const unsigned long long s0 = hE0 & w0, s1 = hE1 & w1;  // attempts
        long long Xc = (rr < n - pos ? rr : n - pos) + __popcll(s0) + __popcll(s1);
        int32_t lc = (pos + rr - 1 < n - 1 ? pos + rr - 1 : n - 1);  // the last gap state's symbol
        const int32_t top1 = s1 ? base + 127 - __clzll(s1) : (s0 ? base + 63 - __clzll(s0) : -1);
        lc = top1 > lc ? top1 : lc;
        bool hit = false;
        if (end0) {
            // E's target is the chain's end: every attempt reports at once.
            hit = (s0 | s1) != 0;
            if (em)
                for (int h = 0; h < 2; ++h)
                    for (unsigned long long m = h ? s1 : s0; m; m &= m - 1)
                        emit_state(c, u0, g.start, base + 64 * h + (__ffsll((long long)m) - 1), k);
        } else if (s0 | s1) {
            // Attempts whose second state is entered (the byte after the
            // first passes the chain's first edge, hT).
            unsigned long long hT0, hT1;
            mask96(c, (uint32_t)gr.lab_off, bm, base, hT0, hT1);
            const unsigned long long d0 = s0 & v0 & ((hT0 >> 1) | (hT1 << 63)), d1 = s1 & v1 & (hT1 >> 1);
            Xc += __popcll(d0) + __popcll(d1);
            if (d0 | d1) {
                const uint32_t u1 = a.rec[u0 & kStateMask].e0_tgt;
                for (int h = 0; h < 2; ++h)
                    for (unsigned long long m = h ? d1 : d0; m; m &= m - 1) {
                        const int32_t p = base + 64 * h + (__ffsll((long long)m) - 1);
                        // The attempt holds u at symbol t; it ends at the
                        // chain's final end or when a byte fails (or the
                        // input ends).
                        uint32_t u = u1;
                        int32_t t = p + 1;
                        for (;;) {
                            if (u & kTgtFinal) {
                                hit = true;
                                if (em) emit_state(c, u, g.start, t, k);
                                break;
                            }
                            if (t + 1 >= n) break;
                            const NfaRec ru = a.rec[u & kStateMask];
                            if (!edge_matches(a, ru.e0_test, c.xa[t + 1])) break;
                            ++Xc;
                            u = ru.e0_tgt;
                            ++t;
                        }
                        lc = t > lc ? t : lc;
                    }
            }
        }
        if (!em) {
            X += Xc;
            last = lc > last ? lc : last;
            if (hit) {
                ++nm;
                qm = w;
            }
        }
    }
    if (nm >= 2) {
        // Replayed by the workgroup from its start: T and X from pos on,
        // reports from the k-th on.
        const int slot = atomicAdd(nbig, 1);
        if (slot < BC) big_s[slot] = Big{g.start, g.k, pos, 0};
        return;
    }
    c.X += X;
    c.T += (last - pos + 2 < n - pos ? last - pos + 2 : n - pos);
}

template <class Ctx>
__device__ __forceinline__ void drain_round(Ctx &c, Walk *q, int &qcount, Big *big_s, int *nbig, GapEnt *gl,
                                            int &gcount) {
    const NfaArgs &a = c.a;
    const int lane = lane_id();
    Walk e[QK];
    bool alive[QK];
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const int idx = lane + 64 * j;
        alive[j] = idx < qcount;
        if (alive[j]) e[j] = q[idx];
        else e[j].n = 0;
    }
    __builtin_amdgcn_wave_barrier();
    uint4 ch[QK];
    int32_t cend[QK];  // end of the walk's chunk (or of the input)
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        cend[j] = 0;
        ch[j] = make_uint4(0, 0, 0, 0);
        if (alive[j]) {
            const int64_t c0 = (int64_t)(e[j].pos & ~15);
            ch[j] = load_granule(c.xa, c0);
            ++c.L;
            cend[j] = (int32_t)(c0 + 16 < c.nP ? c0 + 16 : c.nP);
        }
    }
    // Each pass consumes at least one byte of every active walk, so 16
    // passes finish the chunk.
    for (int st = 0; st < 16; ++st) {
        bool act[QK];
        bool any = false;
#pragma unroll
        for (int j = 0; j < QK; ++j) {
            act[j] = alive[j] && e[j].pos < cend[j];
            any |= act[j];
        }
        if (!__any(any)) break;
        NfaRec r[QK][K];
#pragma unroll
        for (int j = 0; j < QK; ++j)
#pragma unroll
            for (int t = 0; t < K; ++t)
                if (act[j] && t < e[j].n) r[j][t] = a.rec[e[j].s[t] & kStateMask];
        if constexpr (!Ctx::kCarryOn) {
            // A set of gap states whose gaps end in simple chains (once at
            // most 64 any-byte steps remain in each), the chains distinct,
            // waits for a gap pass instead.
#pragma unroll
            for (int j = 0; j < QK; ++j) {
                bool fin = act[j];
#pragma unroll
                for (int t = 0; t < K; ++t)
                    if (t < e[j].n) fin = fin && (r[j][t].info & kRecGapFin) && r[j][t].edge_off <= 64;
#pragma unroll
                for (int t = 1; t < K; ++t)
#pragma unroll
                    for (int t2 = 0; t2 < t; ++t2)
                        if (t < e[j].n) fin = fin && ((r[j][t].e0_tgt ^ r[j][t2].e0_tgt) & kStateMask) != 0;
                const int slot = wave_push_slot(gcount, fin);
                if (fin) {
                    GapEnt *ge = gl + slot;
                    ge->start = e[j].start;
                    ge->pos = e[j].pos;
                    ge->k = e[j].k;
                    ge->n = e[j].n;
#pragma unroll
                    for (int t = 0; t < K; ++t) ge->s[t] = e[j].s[t];
                    act[j] = false;
                    alive[j] = false;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < QK; ++j) {
            if (!act[j]) continue;
            if (e[j].n == 1 && (r[j][0].info & kRecGap)) {
                // A lone gap state: every byte its other edge rejects moves
                // it one state along the gap (one instance-step, one live
                // state, no report), while any-byte steps remain.  Only the
                // walk's chunk is read: loads past it, one lane at a time,
                // cost more than the queue's next round.
                const int32_t room = cend[j] - e[j].pos;  // compared first: pos + edge_off may not fit 32 bits
                const int32_t lim = r[j][0].edge_off < room ? e[j].pos + r[j][0].edge_off : cend[j];
                int32_t p = e[j].pos;
                while (p < lim && !edge_matches(a, r[j][0].e0_test, byte_of(ch[j], p & 15))) ++p;
                const int32_t skip = p - e[j].pos;
                if (skip > 0) {
                    c.T += skip;
                    c.X += skip;
                    e[j].s[0] += (uint32_t)skip;
                    e[j].pos = p;
                    continue;
                }
            }
            uint32_t O[K];
            int nO;
            if (!nfa_step_rec(a, r[j], e[j].n, byte_of(ch[j], e[j].pos & 15), O, nO)) {
                const int slot = atomicAdd(nbig, 1);
                if (slot < BC) big_s[slot] = Big{e[j].start, e[j].k, e[j].pos, 0};
                alive[j] = false;
                continue;
            }
            ++c.T;
            c.X += nO;
            emit_set(c, kBuffer, O, nO, e[j].start, e[j].pos, e[j].k, 0, 0);
#pragma unroll
            for (int t = 0; t < K; ++t) e[j].s[t] = O[t];
            e[j].n = nO;
            ++e[j].pos;
            if (nO == 0) alive[j] = false;
        }
    }
    int nc = 0;
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const bool keep = alive[j] && e[j].n > 0 && e[j].pos < c.n32;
        if (alive[j] && e[j].n > 0 && e[j].pos >= c.n32) c.carry_set(e[j].start, e[j].s, e[j].n);
        const int slot = wave_push_slot(nc, keep);
        if (keep) q[slot] = e[j];
    }
    __builtin_amdgcn_wave_barrier();
    qcount = nc;
    // A round adds at most QW gap walks, so fewer than 64 must wait after it.
    if constexpr (!Ctx::kCarryOn)
        while (gcount >= 64) gap_pass(c, gl, gcount, big_s, nbig);
}

template <bool kCarry>
__global__ __launch_bounds__(NT, 2) void nfa_scan_kernel(NfaArgs a, DfaDefer d) {
    __shared__ uint32_t pbits_s[2048];
    __shared__ int32_t f1o_s[257];
    __shared__ int32_t e1o_s[257];
    __shared__ int16_t n1_s[256];   // states after the first symbol, by byte
    __shared__ int16_t e1n_s[256];  // labels reported after the first symbol, by byte
    __shared__ uint32_t lst_all[(NT / 64) * LC];
    __shared__ Walk qall[(NT / 64) * QW];
    __shared__ uint32_t mkey[MC];
    __shared__ int32_t mend[MC];
    __shared__ int32_t mlab[MC];
    __shared__ Big big_s[BC];
    __shared__ GapEnt gap_all[kCarry ? 1 : (NT / 64) * GC];
    __shared__ int mn, ovf, nbig, seg_s, last_s, nsegs_s, segbase_s;
    __shared__ int sh[16];
    __shared__ long long red[NT / 64];
    __shared__ long long red4[4 * (NT / 64)];
    __shared__ long long ex_s, base_s, segsz_s, dat_s;
    __shared__ int defer_s;
    __shared__ unsigned epoch_s;

    const int tid = threadIdx.x;
    const int wv = tid >> 6;
    const int lane = lane_id();
    const int b = blockIdx.x;
    if (tid == 0) {
        seg_s = take_ticket(a.ctl);
        epoch_s = lb_epoch(a.ctl);
        nsegs_s = a.plan.n_segs_dev ? *a.plan.n_segs_dev : a.n_segs;
        segbase_s = a.plan.seg_base_dev ? *a.plan.seg_base_dev : 0;
        base_s = a.plan.base_dev ? *a.plan.base_dev : 0;
        segsz_s = a.plan.seg_dev ? *a.plan.seg_dev : a.seg;
        mn = 0;
        ovf = 0;
        nbig = 0;
    }
    __syncthreads();
    const int n_segs = nsegs_s;
    if (seg_s >= n_segs) {
        if (n_segs == 0 && b == 0 && tid == 0) *a.total = base_s;
        if (tid == 0) a.bstats[4 * b] = a.bstats[4 * b + 1] = a.bstats[4 * b + 2] = a.bstats[4 * b + 3] = 0;
        finish_launch<NT>(a.ctl, a.lb, a.lb_cap, &last_s);
        return;
    }
    const int seg_base = segbase_s;
    const long long out_base = base_s;
    const int64_t seg_bytes = segsz_s;
    if (a.pair_on)
        for (int i = tid; i < 2048; i += NT) pbits_s[i] = a.p_bits[i];
    for (int i = tid; i < 257; i += NT) {
        f1o_s[i] = a.f1_off[i];
        e1o_s[i] = a.e1_off[i];
    }
    __syncthreads();
    for (int i = tid; i < 256; i += NT) {
        const int n1 = f1o_s[i + 1] - f1o_s[i], e1 = e1o_s[i + 1] - e1o_s[i];
        n1_s[i] = (int16_t)(n1 < 32767 ? n1 : 32767);
        e1n_s[i] = (int16_t)(e1 < 32767 ? e1 : 32767);
    }
    __syncthreads();
    const unsigned epoch = epoch_s;
    const size_t ns = (size_t)a.n_states;
    uint32_t *F0 = a.big_front + (size_t)b * 2 * ns;
    uint32_t *F1 = F0 + ns;
    uint32_t *bits = a.big_bits + (size_t)b * ((ns + 31) / 32);

    NfaCtx<kCarry> c{a, pbits_s, f1o_s, e1o_s, mkey, mend, mlab, &mn, &ovf};
    constexpr bool cy = kCarry;
    Walk *q = qall + wv * QW;
    uint32_t *lst = lst_all + wv * LC;
    GapEnt *gl = kCarry ? gap_all : gap_all + wv * GC;
    int gcount = 0;

    // Replay every listed start with the whole workgroup.
    auto run_big = [&]() __attribute__((always_inline)) {
        __syncthreads();
        const int nb = min(nbig, BC);
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            const Big bg = big_s[j];
            walk_block(c, bg.start, bg.k0, bg.pos0, kBuffer, 0, F0, F1, bits, sh);
        }
        __syncthreads();
        // Starts dropped from a full list are walked by nobody: the segment
        // is then recounted and rewritten from per-start walks.
        if (tid == 0) {
            if (nbig > BC) ovf = 1;
            nbig = 0;
        }
        __syncthreads();
    };
    // Replay the listed starts once the list is half full (a uniform
    // decision taken at the end of every fourth window: each check holds
    // the workgroup's waves until the slowest arrives).  Returns the number
    // of listed starts seen.
    auto replay_if_full = [&](int &qcount) __attribute__((always_inline)) {
        __syncthreads();
        const int pending = nbig;
        __syncthreads();
        if (pending > BC / 2) {
            while (qcount > 0) drain_round(c, q, qcount, big_s, &nbig, gl, gcount);
            run_big();
        }
        return pending;
    };

    for (;;) {
        const int sg = seg_s;
        if (sg >= n_segs) break;
        const uint8_t *sx;
        int64_t sn, seg_lo;
        int stream;
        seg_resolve(a.plan, a.x, a.n, seg_bytes, sg, seg_base, sx, sn, seg_lo, stream);
        const int64_t seg_hi = seg_lo + seg_bytes < sn ? seg_lo + seg_bytes : sn;
        // Shifted positions: p = stream position + dsh, byte p of xa.
        const int dsh = (int)(reinterpret_cast<uintptr_t>(sx) & 15);
        c.xa = sx - dsh;
        c.dsh = dsh;
        c.nP = sn + dsh;
        c.n32 = (int32_t)c.nP;
        const int32_t n32 = c.n32;
        const int64_t own_lo = seg_lo + dsh, own_hi = seg_hi + dsh;
        c.seg_lo = own_lo;
        const long long m_before = c.M, t_before = c.T, x_before = c.X;
        int qcount = 0;
        int lcount = 0;  // entries in the wave's list
        bool checking = true;
        for (int64_t wbase = own_lo & ~(int64_t)15; wbase < own_hi; wbase += W) {
            const int64_t i0 = wbase + 16 * tid;
            const uint4 mine = i0 < c.nP ? load_granule(c.xa, i0) : make_uint4(0, 0, 0, 0);
            // Starts owned by this thread: its 16 bytes within [own_lo, own_hi).
            const int64_t hi64 = own_hi - i0, lo64 = own_lo - i0;
            const int khi = hi64 <= 0 ? 0 : (hi64 >= 16 ? 16 : (int)hi64);
            const int klo = lo64 <= 0 ? 0 : (lo64 >= 16 ? 16 : (int)lo64);
            const unsigned vmask = ((1u << khi) - 1u) & ~((1u << klo) - 1u);
            const int tail = ((vmask >> 15) & 1u) && i0 + 16 < c.nP ? c.xa[i0 + 16] : 0;
            // Every start takes its first symbol (and, when the byte pair has
            // neither states nor labels after two symbols, its second) in
            // registers; the others are appended to the wave's list, which
            // is taken 64 entries at a time as it fills (the rest at the
            // segment's last window), so that every batch of dependent loads
            // serves a full wave.
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                unsigned lm = 0;
                uint32_t ent8[8];
#pragma unroll
                for (int k8 = 0; k8 < 8; ++k8) {
                    const int k = 8 * h + k8;
                    const int32_t i = (int32_t)(i0 + k);
                    const int c1 = byte_of(mine, k);
                    const int c2 = k < 15 ? byte_of(mine, k + 1) : tail;
                    const int n1 = n1_s[c1];
                    const int e1 = e1n_s[c1];
                    const int p = (c1 << 8) | c2;
                    const bool pb = !a.pair_on || ((pbits_s[p >> 5] >> (p & 31)) & 1u);
                    const bool valid = (vmask >> k) & 1u;
                    const bool second = valid && n1 > 0 && i + 1 < n32;
                    // (with carries collected, the last start is listed too:
                    // its first set is live at the end of the input)
                    const bool take = valid && n1 > 0 && (e1 > 0 || (second && pb) || (cy && !second));
                    c.T += valid ? 1 : 0;
                    c.X += valid ? n1 : 0;
                    c.T += (second && !take) ? 1 : 0;
                    lm |= (take ? 1u : 0u) << k8;
                    ent8[k8] = (uint32_t)(i - own_lo) | ((uint32_t)c1 << 16) | ((uint32_t)c2 << 24);
                }
                const int cnt = __popc(lm);
                int total;
                const int ex = wave_excl_small(cnt, total);
                // Every candidate is written: listed starts at their rank, the
                // others past them (fewer than 64 entries wait before a half
                // is added, so the list's last slot is free unless every
                // candidate is listed, and then none is dropped).
                const int spare = lcount + total + lane < LC - 1 ? lcount + total + lane : LC - 1;
#pragma unroll
                for (int k8 = 0; k8 < 8; ++k8)
                    lst[((lm >> k8) & 1u) ? lcount + ex + __popc(lm & ((1u << k8) - 1u)) : spare] = ent8[k8];
                lcount += total;
                __builtin_amdgcn_wave_barrier();
                const bool last = h == 1 && wbase + W >= own_hi;
                for (;;) {
                    const int nb = lcount >= 64 ? 64 : (last ? lcount : 0);
                    if (nb == 0) break;
                    const int e = lane;
                    bool push = false;
                    Walk ent;
                    ent.n = 0;
                    if (e < nb) {
                        const uint32_t w = lst[e];
                        const int32_t i = (int32_t)(own_lo + (w & 0xffffu));
                        const int c1 = (int)((w >> 16) & 255u), c2 = (int)(w >> 24);
                        int32_t km = 0;
                        emit_list(c, kBuffer, a.e1, e1o_s[c1], e1o_s[c1 + 1], i, i, km, 0, 0);
                        if (i + 1 < n32) {
                            int llo, lhi;
                            bool over;
                            const int nS = first_two(c, c1, c2, ent.s, llo, lhi, over);
                            if (over) {
                                const int slot = atomicAdd(&nbig, 1);
                                if (slot < BC) big_s[slot] = Big{i, km, i + 1, 0};
                            } else {
                                ++c.T;
                                c.X += nS;
                                if (a.pair_on) emit_list(c, kBuffer, a.p_lab, llo, lhi, i, i + 1, km, 0, 0);
                                else emit_set(c, kBuffer, ent.s, nS, i, i + 1, km, 0, 0);
                                if (nS > 0 && i + 2 < n32) {
                                    // Symbol three here: most of these walks
                                    // end at it, and only the others queue.
                                    uint32_t O[K];
                                    int nO;
                                    if (!nfa_step(a, ent.s, nS, c.xa[i + 2], O, nO)) {
                                        const int slot = atomicAdd(&nbig, 1);
                                        if (slot < BC) big_s[slot] = Big{i, km, i + 2, 0};
                                    } else {
                                        ++c.T;
                                        c.X += nO;
                                        emit_set(c, kBuffer, O, nO, i, i + 2, km, 0, 0);
                                        if (nO > 0 && i + 3 < n32) {
                                            push = true;
                                            ent.start = i;
                                            ent.pos = i + 3;
                                            ent.k = km;
                                            ent.n = nO;
#pragma unroll
                                            for (int t = 0; t < K; ++t) ent.s[t] = O[t];
                                        } else if (nO > 0) {
                                            c.carry_set(i, O, nO);
                                        }
                                    }
                                } else if (nS > 0) {
                                    c.carry_set(i, ent.s, nS);
                                }
                            }
                        } else {
                            c.carry_first(i, c1);
                        }
                    }
                    while (qcount > QW - 64) drain_round(c, q, qcount, big_s, &nbig, gl, gcount);
                    const int slot = wave_push_slot(qcount, push);
                    if (push) q[slot] = ent;
                    // the batch leaves the list
                    __builtin_amdgcn_wave_barrier();
                    for (int m = nb + lane; m < lcount; m += 64) lst[m - nb] = lst[m];
                    __builtin_amdgcn_wave_barrier();
                    lcount -= nb;
                }
            }
            // The segment's end replays anyway; a segment whose list stays
            // short by its first check stops checking.
            if ((((wbase - (own_lo & ~(int64_t)15)) / W) & 3) == 3 && wbase + W < own_hi && checking)
                checking = replay_if_full(qcount) > BC / 8;
        }
        while (qcount > 0) drain_round(c, q, qcount, big_s, &nbig, gl, gcount);
        if constexpr (!kCarry)
            while (gcount > 0) gap_pass(c, gl, gcount, big_s, &nbig);
        __syncthreads();
        if (nbig > BC) {
            // more starts overflowed than the list holds: the whole segment
            // is rebuilt below from per-start walks
            if (tid == 0) ovf = 1;
        }
        __syncthreads();
        if (!ovf) run_big();
        __syncthreads();
        long long seg_m = c.M - m_before;
        if (ovf) {
            // Starts were dropped from the replay list (or matches did not
            // fit): the segment's count and work come from fresh walks of
            // every owned start.
            c.T = t_before;
            c.X = x_before;
            seg_m = 0;
            for (int64_t c0 = own_lo; c0 < own_hi; c0 += NT) {
                const int64_t i = c0 + tid;
                long long cnt = i < own_hi ? walk_lane(c, (int32_t)i, kCount, 0, true) : 0;
                for (;;) {
                    const int want = block_min(cnt < 0 ? tid : 0x7fffffff, sh + 1);
                    if (want == 0x7fffffff) break;
                    const long long v = walk_block(c, (int32_t)(c0 + want), 0, 0, kCount, 0, F0, F1, bits, sh);
                    if (tid == want) cnt = v;
                    __syncthreads();
                }
                seg_m += cnt;
            }
            c.M = m_before + seg_m;
        }

        // The segment's count, then its placement: staged for a follow-up
        // launch (plain scans, as in the DFA scan), or at the offset found by
        // look-back.
        const long long mine_m = block_sum<NT>(seg_m, red);
        if (tid == 0) {
            seg_s = take_ticket(a.ctl);  // the next segment, requested early
            defer_s = 0;
            if (d.stage && !ovf) {
                const long long at = mine_m ? (long long)atomicAdd(d.cursor, (unsigned long long)mine_m) : 0;
                if (at + mine_m <= d.stage_cap) {
                    defer_s = 1;
                    dat_s = at;
                }
            }
        }
        __syncthreads();
        const bool defer = defer_s != 0;
        if (defer) {
            // Publish the count and go on: the offset comes later.
            if (tid == 0) {
                d.seg_at[sg] = dat_s;
                d.seg_cnt[sg] = mine_m;
                slot_store(&a.lb[sg], lb_pack(epoch, sg == 0 ? kLbIncl : kLbAgg, mine_m));
            }
        } else if (wv == 0) {
            const long long ex = lookback(a.lb, sg, epoch, mine_m);
            if (lane == 0) {
                if (d.stage) {
                    d.seg_at[sg] = -1;
                    d.seg_cnt[sg] = mine_m;
                }
                ex_s = ex;
                const long long at = out_base + ex;
                if (sg == n_segs - 1) *a.total = at + mine_m;
                if (stream >= 0) {
                    if (seg_lo == 0) a.plan.stream_lo[stream] = at;
                    if (seg_hi == sn) a.plan.stream_hi[stream] = at + mine_m;
                }
            }
        }
        __syncthreads();
        const long long at0 = out_base + ex_s;
        if (!ovf) {
            const int m = mn;
            for (int e = tid; e < m; e += NT) {
                const uint32_t mk = mkey[e];
                int rank = 0;
                int j = 0;
                for (; j + 16 <= m; j += 16) {
                    const uint4 k0 = *reinterpret_cast<const uint4 *>(mkey + j);
                    const uint4 k1 = *reinterpret_cast<const uint4 *>(mkey + j + 4);
                    const uint4 k2 = *reinterpret_cast<const uint4 *>(mkey + j + 8);
                    const uint4 k3 = *reinterpret_cast<const uint4 *>(mkey + j + 12);
                    rank += (k0.x < mk) + (k0.y < mk) + (k0.z < mk) + (k0.w < mk);
                    rank += (k1.x < mk) + (k1.y < mk) + (k1.z < mk) + (k1.w < mk);
                    rank += (k2.x < mk) + (k2.y < mk) + (k2.z < mk) + (k2.w < mk);
                    rank += (k3.x < mk) + (k3.y < mk) + (k3.z < mk) + (k3.w < mk);
                }
                for (; j < m; ++j) rank += mkey[j] < mk;
                const long long at = defer ? dat_s + rank : at0 + rank;
                if (defer || at < a.cap) {
                    MatchOut *p = defer ? &d.stage[at] : &a.out[at];
                    p->start = (int32_t)(seg_lo + (mk >> 16));  // stream position
                    p->end = mend[e];
                    p->label = mlab[e];
                }
            }
        } else {
            // Dense segment: count, scan and write 256 starts at a time.
            long long run = at0;
            for (int64_t c0 = own_lo; c0 < own_hi; c0 += NT) {
                const int64_t i = c0 + tid;
                const bool own = i < own_hi;
                long long cnt = own ? walk_lane(c, (int32_t)i, kCount, 0) : 0;
                // starts whose sets outgrow K: counted by the whole workgroup
                for (;;) {
                    const int want = block_min(cnt < 0 ? tid : 0x7fffffff, sh + 1);
                    if (want == 0x7fffffff) break;
                    const long long v =
                        walk_block(c, (int32_t)(c0 + want), 0, 0x7fffffff, kCount, 0, F0, F1, bits, sh);
                    if (tid == want) cnt = v;
                    __syncthreads();
                }
                long long ctot;
                const long long ex = block_excl_scan<NT>(cnt, red, &ctot);
                const long long lane_cnt = own && cnt > 0 ? walk_lane(c, (int32_t)i, kWrite, run + ex) : 0;
                bool pend = lane_cnt < 0;
                for (;;) {
                    const int want = block_min(pend ? tid : 0x7fffffff, sh + 1);
                    if (want == 0x7fffffff) break;
                    if (tid == want) red[0] = run + ex;
                    __syncthreads();
                    const long long base = red[0];
                    __syncthreads();
                    walk_block(c, (int32_t)(c0 + want), 0, 0x7fffffff, kWrite, base, F0, F1, bits, sh);
                    if (tid == want) pend = false;
                }
                __syncthreads();
                run += ctot;
            }
        }
        __syncthreads();
        if (tid == 0) {
            mn = 0;
            ovf = 0;
            nbig = 0;
        }
        __syncthreads();
    }
    long long st4[4] = {c.T, c.X, c.L, c.M};
    block_sum4<NT>(st4, red4);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.bstats[4 * b + k] = st4[k];
    }
    finish_launch<NT>(a.ctl, a.lb, a.lb_cap, &last_s);
}

// Carried instances through a piece, one workgroup per instance: its state
// set becomes the workgroup's frontier, which advances one byte at a time as
// in a replay.  Count pass: matches per instance, and the instances still
// live after the piece go to the carry list; write pass: the matches, in
// (end, label) order, from the instance's output offset on.
__global__ __launch_bounds__(NT) void nfa_resume_kernel(NfaResumeArgs r) {
    __shared__ int sh[16];
    const NfaArgs &a = r.a;
    const int tid = threadIdx.x;
    const size_t ns = (size_t)a.n_states;
    uint32_t *F0 = a.big_front + (size_t)blockIdx.x * 2 * ns;
    uint32_t *F1 = F0 + ns;
    uint32_t *bits = a.big_bits + (size_t)blockIdx.x * ((ns + 31) / 32);
    const int G = *r.in.n_groups;
    if (tid == 0) sh[0] = 0;
    __syncthreads();
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const int k0 = r.in.grp_off[g], k1 = r.in.grp_off[g + 1];
        const int32_t start = (int32_t)(r.in.keys[k0] >> 32);
        int nF = k1 - k0;
        for (int j = tid; j < nF; j += NT) F0[j] = (uint32_t)r.in.keys[k0 + j];
        __syncthreads();
        const long long at = r.write ? r.off[g] : 0;
        long long k = 0;  // tracked by every thread identically
        uint32_t *cur = F0, *nxt = F1;
        for (int64_t p = 0; p < a.n && nF > 0; ++p) {
            const int nN = frontier_step(a, cur, nF, a.x[p], nxt, bits, sh);
            frontier_labels(a, nxt, nN, sh, [&](int m) {
                if (r.write && tid == 0 && at + k < a.cap) {
                    MatchOut *o = &a.out[at + k];
                    o->start = start;
                    o->end = r.base + (int32_t)p;
                    o->label = m;
                }
                ++k;
            });
            uint32_t *t = cur;
            cur = nxt;
            nxt = t;
            nF = nN;
            __syncthreads();
        }
        if (!r.write) {
            if (tid == 0) r.cnt[g] = k;
            for (int j = tid; j < nF; j += NT)
                carry_write(a.carry, carry_reserve(a.carry, 1), start - a.carry.base, cur[j] & kStateMask);
        }
        __syncthreads();
    }
}

}  // namespace

const void *nfa_kernel_fn(bool carry) {
    return carry ? reinterpret_cast<const void *>(&nfa_scan_kernel<true>)
                 : reinterpret_cast<const void *>(&nfa_scan_kernel<false>);
}

hipError_t launch_nfa_resume(const NfaResumeArgs &r, int grid, hipStream_t s) {
    hipLaunchKernelGGL(nfa_resume_kernel, dim3(grid), dim3(NT), 0, s, r);
    return hipGetLastError();
}

}  // namespace pfsmk
