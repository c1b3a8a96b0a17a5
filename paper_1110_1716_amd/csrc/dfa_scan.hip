// All-matches DFA scan for gfx950 (Section III.B with a deterministic
// transition function; the DFA case of Section III.C).
//
// An ordinary launch of 768-thread workgroups (12 wave64, one per compute
// unit when the table is resident in LDS), at most as many as fit at once.
// Workgroups take segments of the input from a ticket counter; a segment
// owns its start positions and its walks read past its end until they die
// (lazy data partitioning, Section III.D.2).  Within a segment the waves
// take 1 KiB slices (16 bytes per lane) from an LDS counter, with no other
// synchronisation between waves:
//   1. the wave stages its slice and the next 1 KiB in a private 2 KiB LDS
//      ring;
//   2. every start takes its first symbol through a byte-indexed liveness
//      table of q0's row (Section III.B steps 1-4 for the fresh tag), 16
//      independent lookups per lane; the starts that survive are compacted
//      (ballot prefix) into a list and walk on through the table (resident
//      in LDS, or the LDS copies of q0's successor rows) with every lane
//      busy, one LDS round trip per step;
//   3. a walk that reaches the end of the staged pair waits in a
//      wave-private LDS queue, and the queued walks finish at the end of
//      the slice, reading through L2 in 16-byte chunks;
//   4. every final state entered adds (start, end, label) to an LDS buffer
//      under the key (start - segment start, k), k = the instance's match
//      count so far, which orders (end, label) within a start (Section III.B
//      reporting rule).
// At the end of a segment the workgroup publishes its match count.  In a
// plain scan of enough segments it then writes its buffered matches, at
// their ranks, to staging rows and moves on; a follow-up launch places them
// (dfa_defer.h).  Otherwise it finds its output offset by decoupled
// look-back over earlier tickets (a predecessor holds an earlier ticket, so
// it is already running) and writes every buffered match at its rank.  A
// segment whose matches do not fit the buffer, or whose parked walks
// outgrow the spill area, is re-walked 768 starts at a time: count, scan,
// write.
#include "dfa_defer.h"
#include "scan_common.h"
#include "stream.h"

namespace pfsmk {

namespace {

constexpr int NT = kDfaThreads;
constexpr int WIN = kDfaWin;
constexpr int RING = kDfaRing;
constexpr int QW = kDfaQueue;
constexpr int QK = QW / 64;
constexpr int MC = kDfaMatchCap;

struct QEnt {
    int32_t start, state, pos, k;
};

template <int ENC, bool kId>
struct DfaCtx {
    const DfaArgs &a;
    const uint8_t *xs;
    const uint16_t *f16_s;
    const int16_t *slot_s;
    const int16_t *b2s_s;
    const uint8_t *flags_s;
    const int32_t *laboff_s;
    const int32_t *lab_s;
    const uint8_t *tab_s;
    uint32_t *mkey;
    int32_t *mend;
    int32_t *mlab;
    int *mn;
    int *ovf;
    int64_t sl = 0;       // first byte of the wave's slice (ring offsets are relative to it)
    int32_t sl32 = 0;
    int64_t wbase = 0;    // current window
    int staged = 0;       // bytes staged from wbase (at most RING)
    int64_t seg_lo = 0;   // the segment's first start (shifted position)
    int32_t n32 = 0;      // end of the stream (shifted position)
    // The stream being scanned: positions inside the kernel are shifted by
    // dsh = the stream's offset from the 16-byte boundary below it, so that
    // position p is byte p of the aligned base xa (reported positions are
    // p - dsh).
    const uint8_t *xa = nullptr;
    int64_t nP = 0;
    int32_t dsh = 0;
    long long T = 0, X = 0, L = 0, M = 0;

    static constexpr bool kResident = ENC == kEnc8 || ENC == kEnc8D || ENC == kEnc16;

    __device__ __forceinline__ uint8_t flag(int s) const {
        if constexpr (kResident) return flags_s[s];
        else return a.flags[s];
    }
    __device__ __forceinline__ int sym(int byte) const { return kId ? byte : (int)b2s_s[byte]; }
    // Live target of q0 on byte b, or -1.  States below 2^15 come from the
    // 16-bit row in LDS, larger ones from the row in memory.
    __device__ __forceinline__ int first_state(int b) const {
        if constexpr (ENC == kCold32) {
            return a.first[b];
        } else {
            const unsigned v = f16_s[b];
            return (v & 0x8000u) ? (int)(v & 0x7fffu) : -1;
        }
    }
    // delta(s, sy) as given: a state or -1.
    __device__ __forceinline__ int tab(int s, int sy) const {
        if constexpr (ENC == kEnc8) {
            const int v = tab_s[(uint32_t)s * (uint32_t)a.n_symbols + (uint32_t)sy];
            return v == 255 ? -1 : v;
        } else if constexpr (ENC == kEnc8D) {
            // 256 states: the byte and its dead bit are read side by side.
            const uint32_t i = ((uint32_t)s << 8) | (uint32_t)sy;
            const uint32_t *dead = reinterpret_cast<const uint32_t *>(tab_s + 65536);
            const int v = tab_s[i];
            const uint32_t w = dead[i >> 5];
            return (w >> (i & 31)) & 1u ? -1 : v;
        } else if constexpr (ENC == kEnc16) {
            return reinterpret_cast<const int16_t *>(tab_s)[(uint32_t)s * (uint32_t)a.n_symbols + (uint32_t)sy];
        } else if constexpr (ENC == kCold16) {
            return reinterpret_cast<const int16_t *>(a.tbl)[(int64_t)s * a.n_symbols + sy];
        } else {
            return reinterpret_cast<const int32_t *>(a.tbl)[(int64_t)s * a.n_symbols + sy];
        }
    }
    // delta(s, sy) read without branches (s and sy in range): the reads of a
    // step can then be issued together.
    __device__ __forceinline__ int tab_any(int s, int sy) const {
        if constexpr (ENC == kEnc8D) {
            const uint32_t i = ((uint32_t)s << 8) | (uint32_t)sy;
            const uint32_t *dead = reinterpret_cast<const uint32_t *>(tab_s + 65536);
            const int v = tab_s[i];
            const uint32_t w = dead[i >> 5];
            return ((w >> (i & 31)) & 1u) ? -1 : v;
        } else {
            return tab(s, sy);
        }
    }
    // Second symbol of a walk whose first step read byte b0 and reached s1.
    __device__ __forceinline__ int tab2(int b0, int s1, int sy) const {
        if constexpr (kResident) {
            return tab(s1, sy);
        } else {
            const int slot = slot_s[b0];
            if (slot < 0) return tab(s1, sy);
            if constexpr (ENC == kCold16) return reinterpret_cast<const int16_t *>(tab_s)[slot * a.n_symbols + sy];
            else return reinterpret_cast<const int32_t *>(tab_s)[slot * a.n_symbols + sy];
        }
    }
    __device__ __forceinline__ int live(int t) const { return (t >= 0 && (flag(t) & kLive)) ? t : -1; }
    __device__ __forceinline__ int lab_lo(int s) const {
        if constexpr (kResident) return laboff_s[s];
        else return a.lab_off[s];
    }
    __device__ __forceinline__ int lab_at(int l) const {
        if constexpr (kResident) return lab_s[l];
        else return a.lab[l];
    }
    // Report every label of s for the instance started at `start`; k counts
    // the instance's reports (ordering key within a start).
    __device__ __forceinline__ void emit(int32_t start, int32_t end, int s, int32_t &k) {
        const int lo = lab_lo(s), cnt = lab_lo(s + 1) - lo;
        M += cnt;
        if (!*ovf) {
            const int slot = atomicAdd(mn, cnt);
            if (slot + cnt <= MC) {
                for (int l = 0; l < cnt; ++l) {
                    mkey[slot + l] = ((uint32_t)(start - seg_lo) << 16) | (uint32_t)((k + l) & 0xffff);
                    mend[slot + l] = end - dsh;
                    mlab[slot + l] = lab_at(lo + l);
                }
            } else {
                *ovf = 1;
            }
        }
        k += cnt;
    }
    __device__ __forceinline__ int n_labels(int s) const { return lab_lo(s + 1) - lab_lo(s); }
    // The instance started at `start` is in live state s after the last byte
    // of the input: hand it to the next piece when carries are collected.
    __device__ __forceinline__ void carry(int32_t start, int s) const {
        if (a.carry.pairs) carry_write(a.carry, carry_reserve(a.carry, 1), start - dsh, (uint32_t)s);
    }
    // The ring byte of position p (meaningful when p is staged; any p reads
    // inside the ring).
    __device__ __forceinline__ int ring_at(int32_t p) const { return xs[(uint32_t)(p - sl32) & (RING - 1)]; }
    // Whether the 16-byte chunk at p (a multiple of 16) is staged in LDS.
    __device__ __forceinline__ bool staged_at(int64_t p) const {
        const int64_t r = p - wbase;
        return r >= 0 && r + 16 <= staged;
    }
    // The 16-byte chunk holding position p (p is a multiple of 16).
    __device__ __forceinline__ uint4 chunk(int64_t p) {
        if (staged_at(p)) return *reinterpret_cast<const uint4 *>(xs + ((p - sl) & (RING - 1)));
        ++L;
        return load_granule(xa, p);
    }
};

// One round: every walk in this wave's queue advances through the rest of
// the 16-byte chunk holding its next position (up to 16 symbols); walks that
// end are dropped and the queue is re-packed.  With kStagedOnly a walk whose
// chunk is not staged in LDS stays where it is.  Returns whether some kept
// walk can advance inside the staged window.
//
// A step issues the reads of both walks of a lane (the flag of the state just
// entered and the table entry of the next symbol) before it uses any of
// them, so the step costs one LDS round trip; reports go through a branch
// that is taken only when some walk of the wave enters a final state.
template <bool kStagedOnly, int ENC, bool kId>
__device__ __forceinline__ bool drain_round(DfaCtx<ENC, kId> &c, QEnt *q, int &qcount) {
    const int lane = lane_id();
    QEnt e[QK];
    bool alive[QK];
    uint4 ch[QK];
    int steps[QK];
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const int idx = lane + 64 * j;
        alive[j] = idx < qcount;
        e[j] = alive[j] ? q[idx] : QEnt{0, 0, 0, 0};
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const int64_t c0 = (int64_t)(e[j].pos & ~15);
        const bool go = alive[j] && (!kStagedOnly || c.staged_at(c0));
        ch[j] = go ? c.chunk(c0) : make_uint4(0, 0, 0, 0);
        const int64_t end = c0 + 16 < c.nP ? c0 + 16 : c.nP;
        steps[j] = go ? (int)(end - e[j].pos) : 0;  // symbols left in this chunk
    }
    // t[j]: target of the walk's next symbol (-1: none), looked up a step ahead.
    int t[QK];
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const int sy = c.sym(byte_of(ch[j], e[j].pos & 15));
        const int v = c.tab_any(e[j].state, sy < 0 ? 0 : sy);
        t[j] = (steps[j] > 0 && sy >= 0) ? v : -1;
    }
#pragma unroll 1
    for (int st = 0; st < 16; ++st) {
        uint8_t f[QK];
        int nx[QK];
#pragma unroll
        for (int j = 0; j < QK; ++j) {
            const int cur = t[j] < 0 ? 0 : t[j];
            f[j] = c.flag(cur);
            const int sy = c.sym(byte_of(ch[j], (e[j].pos + 1) & 15));
            const int v = c.tab_any(cur, sy < 0 ? 0 : sy);
            nx[j] = (sy >= 0 && st + 1 < steps[j]) ? v : -1;
        }
        bool more = false, fin[QK], anyfin = false;
#pragma unroll
        for (int j = 0; j < QK; ++j) {
            const bool act = st < steps[j];
            const bool ok = act && t[j] >= 0 && (f[j] & kLive);
            c.T += act ? 1 : 0;
            c.X += ok ? 1 : 0;
            fin[j] = ok && (f[j] & kFinal);
            anyfin |= fin[j];
            if (act && !ok) steps[j] = 0;  // the walk ends here
            alive[j] = alive[j] && (!act || ok);
            e[j].state = ok ? t[j] : e[j].state;
            e[j].pos += ok ? 1 : 0;
            t[j] = nx[j];
            more |= ok && st + 1 < steps[j];
        }
        if (__any(anyfin)) {
#pragma unroll
            for (int j = 0; j < QK; ++j)
                if (fin[j]) c.emit(e[j].start, e[j].pos - 1, e[j].state, e[j].k);
        }
        if (!__any(more)) break;
    }
    int nc = 0;
    bool again = false;
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const bool keep = alive[j] && e[j].pos < c.n32;
        if (alive[j] && e[j].pos >= c.n32) c.carry(e[j].start, e[j].state);
        again |= keep && c.staged_at((int64_t)(e[j].pos & ~15));
        const int slot = wave_push_slot(nc, keep);
        if (keep) q[slot] = e[j];
    }
    __builtin_amdgcn_wave_barrier();
    qcount = nc;
    return __any(again);
}

// Advances the lane's walk (state s, next position pos) while its bytes are
// staged: it enters states until one is not live or a byte has no
// transition, the input ends, or the staged pair ends at `lim`.  Returns
// whether the walk is still live at `lim` (it then continues in the next
// window).  One LDS round trip per symbol: the flag of the state just
// entered, the table entry of the byte after it and the byte after that are
// read together, before any of them is used.
template <int ENC, bool kId>
__device__ __forceinline__ bool advance_staged(DfaCtx<ENC, kId> &c, bool act, int32_t start, int &s, int32_t &pos,
                                               int32_t &k, int32_t lim) {
    bool run = act && pos < lim;
    bool alive = act;
    int b0 = c.ring_at(pos);
    int bn = c.ring_at(pos + 1);
    int sy = c.sym(b0);
    int t = c.tab_any(s, sy < 0 ? 0 : sy);
    if (sy < 0) t = -1;
    int nT = 0, nX = 0;
    while (__any(run)) {
        const int cur = t < 0 ? 0 : t;
        const uint8_t f = c.flag(cur);
        const int sy2 = c.sym(bn);
        const int tn = c.tab_any(cur, sy2 < 0 ? 0 : sy2);
        const int bnn = c.ring_at(pos + 2);
        const bool ok = run && t >= 0 && (f & kLive);
        nT += run ? 1 : 0;
        nX += ok ? 1 : 0;
        const bool fin = ok && (f & kFinal);
        if (__any(fin)) {
            if (fin) c.emit(start, pos, cur, k);
        }
        if (run && !ok) alive = false;
        s = ok ? cur : s;
        pos += ok ? 1 : 0;
        run = ok && pos < lim;
        t = sy2 < 0 ? -1 : tn;
        bn = bnn;
    }
    c.T += nT;
    c.X += nX;
    if (alive && pos >= c.n32) c.carry(start, s);
    return alive && pos < c.n32;
}

// advance_staged for the 8-bit resident tables with byte-indexed rows.  The
// target of the next byte is carried as the stored byte u and a dead bit d
// (kEnc8: u = 255 marks no transition and its flag entry is zero; kEnc8D: the
// table's dead bit).  A step reads the flag of u, the table entry and dead
// word of (u, next byte) and the byte after, together; the walk's running,
// live and final conditions are kept as 0/1 integers so that a step is
// straight-line vector code.  The walk's counts come from the distance
// walked: X = bytes entered, T adds the killing byte of a walk that ends
// before `lim`.
template <int ENC>
__device__ __forceinline__ bool advance_staged8(DfaCtx<ENC, true> &c, bool act, int32_t start, int &s, int32_t &pos,
                                                int32_t &k, int32_t lim) {
    static_assert(ENC == kEnc8 || ENC == kEnc8D, "8-bit byte-indexed tables only");
    const uint8_t *fl = c.flags_s;
    const uint8_t *tb = c.tab_s;
    const uint32_t *dead = reinterpret_cast<const uint32_t *>(c.tab_s + 65536);
    const uint32_t rmax = (uint32_t)c.a.n_states - 1u;
    const int32_t p0 = pos;
    // Byte p of the staged pair is rb[p - pos].  Running walks read at most
    // two bytes past the pair, which stay inside LDS (the next wave's ring or
    // the fixed head after the last one).
    const uint8_t *rb = c.xs + (uint32_t)(pos - c.sl32);
    const uint8_t *const rb0 = rb;
    const uint8_t *const rlim = rb + (lim - pos);
    // Row index of target u on byte b (kEnc8 rows stop at n_states - 1; the
    // row read for u = 255 is never used).
    auto index = [&](uint32_t u, uint32_t b) __attribute__((always_inline)) -> uint32_t {
        if constexpr (ENC == kEnc8D) return (u << 8) | b;
        else return ((u < rmax ? u : rmax) << 8) | b;
    };
    // Dead bit of table index i in bit 0 of the result (kEnc8: none).
    auto dead_of = [&](uint32_t i) __attribute__((always_inline)) -> uint32_t {
        if constexpr (ENC == kEnc8D) return dead[i >> 5] >> (i & 31);
        else return 0u;
    };
    const uint32_t i0 = index((uint32_t)s, rb[0]);
    uint32_t u = tb[i0];
    uint32_t d = dead_of(i0);
    uint32_t b2 = rb[1];
    const uint32_t r0 = act && rb < rlim ? 1u : 0u;
    uint32_t run = r0;
    while (__any(run != 0)) {
        const uint32_t f = fl[u];
        const uint32_t i = index(u, b2);
        const uint32_t un = tb[i];
        const uint32_t dn = dead_of(i);
        const uint32_t b3 = rb[2];
        // the four reads leave together: nothing below may move above them
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t ok = (run & f) & ~d & 1u;  // flags are 0, kLive or kLive | kFinal
        const uint32_t fin = ok & (f >> 1);
        if (__any(fin != 0)) {
            if (fin) c.emit(start, p0 + (int32_t)(rb - rb0), (int)u, k);
        }
        s = ok ? (int)u : s;
        rb += ok;
        run = rb < rlim ? ok : 0u;
        u = un;
        d = dn;
        b2 = b3;
    }
    const int32_t walked = (int32_t)(rb - rb0);
    pos = p0 + walked;
    // A walk that started is still live exactly when it reached lim.
    const bool alive = act && pos >= lim;
    c.X += walked;
    c.T += r0 ? walked + (alive ? 0 : 1) : 0;
    if (alive && pos >= c.n32) c.carry(start, s);
    return alive && pos < c.n32;
}

// The full walk of one start reading the input through the cache hierarchy;
// counts its matches, or writes them from output index `at` when write.
// With `work`, adds its instance-steps and live steps to work[0] and work[1].
template <int ENC, bool kId>
__device__ __forceinline__ long long walk_start(const DfaCtx<ENC, kId> &c, int32_t i, bool write, long long at,
                                                long long *work = nullptr) {
    const DfaArgs &a = c.a;
    long long cnt = 0, nT = 1, nX = 0;
    int s = c.first_state(c.xa[i]);
    int32_t pos = i;
    if (s >= 0) nX = 1;
    while (s >= 0) {
        for (int l = c.lab_lo(s); l < c.lab_lo(s + 1); ++l, ++cnt) {
            if (write && at + cnt < a.cap) {
                MatchOut *p = &a.out[at + cnt];
                p->start = i - c.dsh;
                p->end = pos - c.dsh;
                p->label = c.lab_at(l);
            }
        }
        if (++pos >= c.n32) {
            if (!write) c.carry(i, s);
            break;
        }
        const int sy = c.sym(c.xa[pos]);
        s = sy < 0 ? -1 : c.live(c.tab(s, sy));
        ++nT;
        nX += s >= 0 ? 1 : 0;
    }
    if (work) {
        work[0] += nT;
        work[1] += nX;
    }
    return cnt;
}

// Move the walks of this wave's queue to the workgroup's spill area in
// memory (stores only).  Returns false when the area is full: the segment is
// then re-walked at its end and the walks are dropped.
__device__ __forceinline__ bool spill_walks(QEnt *q, int &qcount, QEnt *area, int *sp_n) {
    int at = 0;
    if (lane_id() == 0) at = atomicAdd(sp_n, qcount);
    at = __shfl(at, 0);
    const bool fits = at + qcount <= kDfaSpill;
    if (fits)
        for (int e = lane_id(); e < qcount; e += 64) area[at + e] = q[e];
    __builtin_amdgcn_wave_barrier();
    qcount = 0;
    return fits;
}

template <int ENC, bool kId>
__global__ __launch_bounds__(NT) void dfa_scan_kernel(DfaArgs a, DfaDefer d) {
    // States of the 8-bit encodings travel in the live-start list.
    constexpr bool kPack = ENC == kEnc8 || ENC == kEnc8D;
    extern __shared__ __align__(16) uint8_t lds[];
    int16_t *slot_s = reinterpret_cast<int16_t *>(lds + kDfaWaves * RING);
    int16_t *b2s_s = slot_s + 256;
    uint16_t *f16_s = reinterpret_cast<uint16_t *>(b2s_s + 256);
    uint8_t *flags_s = lds + a.off_flags;
    int32_t *laboff_s = reinterpret_cast<int32_t *>(lds + a.off_laboff);
    int32_t *lab_s = reinterpret_cast<int32_t *>(lds + a.off_lab);
    uint8_t *tab_s = lds + a.off_tab;
    QEnt *qall = reinterpret_cast<QEnt *>(lds + a.off_q);
    uint32_t *mkey = reinterpret_cast<uint32_t *>(lds + a.off_m);
    int32_t *mend = reinterpret_cast<int32_t *>(mkey + MC);
    int32_t *mlab = mend + MC;
    __shared__ int mn, ovf, sp_n, seg_s, last_s, slice_s, defer_s;
    __shared__ long long red[NT / 64];
    __shared__ long long red4[4 * (NT / 64)];
    __shared__ long long ex_s, base_s, segsz_s, dat_s;
    __shared__ unsigned epoch_s;
    __shared__ int nsegs_s, segbase_s;

    const int tid = threadIdx.x;
    const int wv = tid >> 6;
    const int lane = lane_id();
    const int b = blockIdx.x;
    uint8_t *ring = lds + wv * RING;
    uint32_t *lst = reinterpret_cast<uint32_t *>(lds + a.off_list) + wv * kDfaList;
    QEnt *spill = reinterpret_cast<QEnt *>(a.spill) + (int64_t)b * kDfaSpill;

    // Every load of the start-up is issued before any is waited for: the LDS
    // image (flags, label CSR, table) in one run of 16-byte loads, q0's row,
    // and the first segment ticket.
    const uint4 *isrc = reinterpret_cast<const uint4 *>(a.res);
    uint4 *idst = reinterpret_cast<uint4 *>(lds + a.off_flags);
    const int n16 = a.res_bytes >> 4;
    int ib = 0;
    for (; ib + 5 * NT < n16; ib += 6 * NT) {
        const uint4 v0 = isrc[ib + tid], v1 = isrc[ib + NT + tid], v2 = isrc[ib + 2 * NT + tid],
                    v3 = isrc[ib + 3 * NT + tid], v4 = isrc[ib + 4 * NT + tid], v5 = isrc[ib + 5 * NT + tid];
        idst[ib + tid] = v0;
        idst[ib + NT + tid] = v1;
        idst[ib + 2 * NT + tid] = v2;
        idst[ib + 3 * NT + tid] = v3;
        idst[ib + 4 * NT + tid] = v4;
        idst[ib + 5 * NT + tid] = v5;
    }
    int fq = -1, fslot = -1, fb = -1;
    if (tid < 256) {
        fq = a.first[tid];
        fslot = a.first_slot[tid];
        fb = a.b2s[tid];
    }
    if (tid == 0) {
        seg_s = take_ticket(a.ctl);
        epoch_s = lb_epoch(a.ctl);
        // Batches: this launch's segment count, list and output base live on
        // the device (written by the planning kernels).
        nsegs_s = a.plan.n_segs_dev ? *a.plan.n_segs_dev : a.n_segs;
        segbase_s = a.plan.seg_base_dev ? *a.plan.seg_base_dev : 0;
        base_s = a.plan.base_dev ? *a.plan.base_dev : 0;
        segsz_s = a.plan.seg_dev ? *a.plan.seg_dev : a.seg;
        mn = 0;
        ovf = 0;
        sp_n = 0;
        slice_s = 0;
    }
    for (int i = ib + tid; i < n16; i += NT) idst[i] = isrc[i];
    if (tid < 256) {
        f16_s[tid] = fq >= 0 ? (uint16_t)(0x8000u | ((unsigned)fq & 0x7fffu)) : (uint16_t)0;
        slot_s[tid] = (int16_t)fslot;
        b2s_s[tid] = (int16_t)fb;
    }
    __syncthreads();
    const int n_segs = nsegs_s;
    if (seg_s >= n_segs) {
        // Nothing to scan: only the launch's bookkeeping remains.
        if (n_segs == 0 && b == 0 && tid == 0) *a.total = base_s;
        if (tid == 0) a.bstats[4 * b] = a.bstats[4 * b + 1] = a.bstats[4 * b + 2] = a.bstats[4 * b + 3] = 0;
        finish_launch<NT>(a.ctl, a.lb, a.lb_cap, &last_s);
        return;
    }
    const int seg_base = segbase_s;
    const long long out_base = base_s;
    const int64_t seg_bytes = segsz_s;
    const unsigned epoch = epoch_s;

    DfaCtx<ENC, kId> c{a, ring, f16_s, slot_s, b2s_s, flags_s, laboff_s, lab_s, tab_s, mkey, mend, mlab, &mn, &ovf};
    QEnt *q = qall + wv * QW;
    int qcount = 0;

    for (;;) {
        const int sg = seg_s;
        if (sg >= n_segs) break;
        // The segment's stream and its range of starts (stream positions).
        const uint8_t *sx;
        int64_t sn, seg_lo;
        int stream;
        seg_resolve(a.plan, a.x, a.n, seg_bytes, sg, seg_base, sx, sn, seg_lo, stream);
        const int64_t seg_hi = seg_lo + seg_bytes < sn ? seg_lo + seg_bytes : sn;
        // Shifted positions: p = stream position + dsh, bytes of xa.
        const int dsh = (int)(reinterpret_cast<uintptr_t>(sx) & 15);
        c.xa = sx - dsh;
        c.dsh = dsh;
        c.nP = sn + dsh;
        c.n32 = (int32_t)c.nP;
        const int32_t n32 = c.n32;
        const int64_t own_lo = seg_lo + dsh, own_hi = seg_hi + dsh;
        const int64_t s0 = own_lo & ~(int64_t)15;
        const long long m_before = c.M, t_before = c.T, x_before = c.X;
        c.seg_lo = own_lo;
        // Waves take the segment's slices (one window each) from a counter,
        // so a wave held by a long walk does not hold the others' work.
        const int n_sl = (int)((own_hi - s0 + WIN - 1) / WIN);
        for (;;) {
        int k_sl = 0;
        if (lane == 0) k_sl = atomicAdd(&slice_s, 1);
        k_sl = __shfl(k_sl, 0);
        if (k_sl >= n_sl) break;
        // The slice owns the starts of [max(sl, own_lo), sh).
        const int64_t sl = s0 + (int64_t)WIN * k_sl;
        const int64_t sh = sl + WIN < own_hi ? sl + WIN : own_hi;
        auto fetch = [&](int64_t wb) __attribute__((always_inline)) {
            const int64_t p = wb + 16 * lane;
            return p < c.nP ? load_granule(c.xa, p) : make_uint4(0, 0, 0, 0);
        };
        // The slice and the next 1 KiB are staged; walks still live at the
        // end of the pair wait in the queue (empty when a slice begins).
        const uint4 cur = fetch(sl);
        const uint4 nxt = sl + WIN < c.nP ? fetch(sl + WIN) : make_uint4(0, 0, 0, 0);
        c.sl = sl;
        c.sl32 = (int32_t)sl;
        *reinterpret_cast<uint4 *>(ring + 16 * lane) = cur;
        *reinterpret_cast<uint4 *>(ring + WIN + 16 * lane) = nxt;
        __builtin_amdgcn_wave_barrier();
        {
            const int64_t wb = sl;
            c.wbase = wb;
            const int64_t rest = c.nP - wb;
            c.staged = (int)(rest < RING ? rest : RING);

            // The staged pair ends at lim.
            const int32_t lim = (int32_t)(rest < RING ? c.nP : wb + RING);

            // Starts owned by this lane: its 16 bytes within [own_lo, sh).
            // (sh - wb and own_lo - wb lie within one segment of each other)
            const int rhi = (int)(sh - wb) - 16 * lane, rlo = (int)(own_lo - wb) - 16 * lane;
            const int khi = rhi <= 0 ? 0 : (rhi >= 16 ? 16 : rhi);
            const int klo = rlo <= 0 ? 0 : (rlo >= 16 ? 16 : rlo);
            const unsigned vmask = ((1u << khi) - 1u) & ~((1u << klo) - 1u);
            c.T += __popc(vmask);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // Symbol one for 8 starts per lane (q0's row by byte), then the
                // list of survivors: offset | state << 10 when states fit 8
                // bits, else the offset alone.
                unsigned lm = 0;
                uint32_t ent8[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const unsigned v = f16_s[byte_of(cur, 8 * h + k)];
                    lm |= (v >> 15) << k;
                    ent8[k] = kPack ? ((uint32_t)(16 * lane + 8 * h + k) | ((v & 0xffu) << 10))
                                    : (uint32_t)(16 * lane + 8 * h + k);
                }
                lm &= (vmask >> (8 * h)) & 0xffu;
                const int cnt = __popc(lm);
                c.X += cnt;
                int total;
                const int ex = wave_excl_small(cnt, total);
                // Every candidate is written: survivors at their rank, the
                // others to a slot past the survivors (the last slot is free
                // unless every candidate survived, and then none is dropped).
                const int spare = total + lane < kDfaList - 1 ? total + lane : kDfaList - 1;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    lst[((lm >> k) & 1u) ? ex + __popc(lm & ((1u << k) - 1u)) : spare] = ent8[k];
                __builtin_amdgcn_wave_barrier();
                for (int e0 = 0; e0 < total; e0 += 64) {
                    const int e = e0 + lane;
                    const bool act = e < total;
                    const uint32_t w = act ? lst[e] : 0u;
                    const int il = (int)(w & 1023u);
                    const int32_t i = (int32_t)(wb + il);
                    int s1 = kPack ? (int)(w >> 10) : c.first_state(c.ring_at(i));
                    if (!act) s1 = 0;
                    int32_t km = 0;
                    if (act && (c.flag(s1) & kFinal)) c.emit(i, i, s1, km);
                    int32_t pos = i + 1;
                    if (act && pos >= n32) c.carry(i, s1);
                    bool park;
                    if constexpr (kId && (ENC == kEnc8 || ENC == kEnc8D))
                        park = advance_staged8(c, act && pos < n32, i, s1, pos, km, lim);
                    else
                        park = advance_staged(c, act && pos < n32, i, s1, pos, km, lim);
                    if (qcount > QW - 64 && __any(park)) {
                        // Too many walks wait for the next window: move them
                        // to memory (they finish at the end of the slice).
                        if (!spill_walks(q, qcount, spill, &sp_n)) ovf = 1;
                    }
                    const int slot = wave_push_slot(qcount, park);
                    if (park) q[slot] = QEnt{i, s1, pos, km};
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        // The slice's walks run to their end (the spilled ones after all
        // slices).
        while (qcount > 0) drain_round<false>(c, q, qcount);
        }
        __syncthreads();
        const int n_sp = ovf ? 0 : sp_n;
        for (int e0 = 64 * wv; e0 < n_sp; e0 += NT) {
            const int e = e0 + lane;
            if (e < n_sp) q[lane] = spill[e];
            qcount = n_sp - e0 < 64 ? n_sp - e0 : 64;
            __builtin_amdgcn_wave_barrier();
            while (qcount > 0) drain_round<false>(c, q, qcount);
        }

        __syncthreads();
        long long seg_m = c.M - m_before;
        if (ovf) {
            // Walks were dropped (or matches did not fit): the segment's
            // count and work come from a fresh walk of every owned start.
            long long work[2] = {0, 0};
            seg_m = 0;
            for (int64_t i = own_lo + tid; i < own_hi; i += NT) seg_m += walk_start(c, (int32_t)i, false, 0, work);
            c.T = t_before + work[0];
            c.X = x_before + work[1];
            c.M = m_before + seg_m;
        }

        // The segment's count, then its placement: staged for a follow-up
        // launch, or at the offset found by look-back.
        const long long mine_m = block_sum<NT>(seg_m, red);
        if (tid == 0) {
            seg_s = take_ticket(a.ctl);  // the next segment, requested early
            // Deferred placement: staging rows for the buffered matches.
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
                    // The stream's range in this launch's output.
                    if (seg_lo == 0) a.plan.stream_lo[stream] = at;
                    if (seg_hi == sn) a.plan.stream_hi[stream] = at + mine_m;
                }
            }
        }
        __syncthreads();
        const long long at0 = out_base + ex_s;
        if (!ovf) {
            // Rank of every buffered match in (start, end, label) order:
            // bucket by start offset / 64 (histogram, scan, scatter), then
            // compare within the bucket.  The queue area is free here.
            const int m = mn;
            int *hist = reinterpret_cast<int *>(qall);
            int *base = hist + 1024;
            int *fill = base + 1024;
            uint32_t *memb = reinterpret_cast<uint32_t *>(fill + 1024);  // keys by bucket
            for (int j = tid; j < 1024; j += NT) {
                hist[j] = 0;
                fill[j] = 0;
            }
            __syncthreads();
            for (int e = tid; e < m; e += NT) atomicAdd(&hist[mkey[e] >> 22], 1);
            __syncthreads();
            int h4[4] = {0, 0, 0, 0};
            long long own = 0;
            if (tid < 256) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    h4[j] = hist[4 * tid + j];
                    own += h4[j];
                }
            }
            long long all_m;
            long long run = block_excl_scan<NT>(own, red, &all_m);
            if (tid < 256) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    base[4 * tid + j] = (int)run;
                    run += h4[j];
                }
            }
            __syncthreads();
            for (int e = tid; e < m; e += NT) {
                const uint32_t mk = mkey[e];
                memb[base[mk >> 22] + atomicAdd(&fill[mk >> 22], 1)] = mk;
            }
            __syncthreads();
            for (int e = tid; e < m; e += NT) {
                const uint32_t mk = mkey[e];
                const int bk = mk >> 22;
                const int lo = base[bk], hi = lo + hist[bk];
                int rank = lo;
                // the bucket's keys, read independently of one another
#pragma unroll 4
                for (int j = lo; j < hi; ++j) rank += memb[j] < mk;
                const long long at = defer ? dat_s + rank : at0 + rank;
                if (defer || at < a.cap) {
                    MatchOut *p = defer ? &d.stage[at] : &a.out[at];
                    p->start = (int32_t)(seg_lo + (mk >> 16));  // stream position
                    p->end = mend[e];
                    p->label = mlab[e];
                }
            }
        } else {
            long long run = at0;
            for (int64_t c0 = own_lo; c0 < own_hi; c0 += NT) {
                const int64_t i = c0 + tid;
                const bool own = i < own_hi;
                const long long cnt = own ? walk_start(c, (int32_t)i, false, 0) : 0;
                long long ctot;
                const long long ex = block_excl_scan<NT>(cnt, red, &ctot);
                if (own && cnt) walk_start(c, (int32_t)i, true, run + ex);
                run += ctot;
            }
        }
        __syncthreads();
        if (tid == 0) {
            mn = 0;
            ovf = 0;
            sp_n = 0;
            slice_s = 0;
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

__global__ void write_zero_kernel(int64_t *p) { *p = 0; }

// Deferred placement in one launch, for launches of at most
// kDeferFusedSegs segments: each workgroup sums the counts before its
// segment, then copies the segment's staged rows (rows at or past `cap` are
// dropped, as in the scan).  The last segment's workgroup writes the total.
__global__ __launch_bounds__(256) void dfa_place_fused_kernel(DfaDefer d, int n_segs, int64_t *total, MatchOut *out,
                                                              int64_t cap) {
    __shared__ long long red[256 / 64];
    const int sg = blockIdx.x;
    long long v = 0;
    for (int i = (int)threadIdx.x; i < sg; i += 256) v += d.seg_cnt[i];
    const long long base = block_sum<256>(v, red);
    const long long cnt = d.seg_cnt[sg];
    if (threadIdx.x == 0) {
        if (sg == n_segs - 1) *total = base + cnt;
        if (sg == 0) *d.cursor = 0;
    }
    const long long at = d.seg_at[sg];
    if (at < 0) return;
    for (long long i = threadIdx.x; i < cnt; i += 256) {
        const long long o = base + i;
        if (o < cap) out[o] = d.stage[at + i];
    }
}

// Deferred placement, first launch: output offsets of the segments (an
// exclusive scan of their counts), the grand total, and the staging counter
// cleared for the next scan on this stream.
__global__ __launch_bounds__(1024) void dfa_place_scan_kernel(DfaDefer d, int n_segs, int64_t *total) {
    __shared__ long long red[1024 / 64];
    long long run = 0;
    for (int c0 = 0; c0 < n_segs; c0 += 1024) {
        const int i = c0 + (int)threadIdx.x;
        const long long v = i < n_segs ? d.seg_cnt[i] : 0;
        long long tot;
        const long long ex = block_excl_scan<1024>(v, red, &tot);
        if (i < n_segs) d.seg_base[i] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        *total = run;
        *d.cursor = 0;
    }
}

// Deferred placement, second launch: staged rows to their output positions
// (rows at or past `cap` are dropped, as in the scan).
__global__ __launch_bounds__(256) void dfa_place_copy_kernel(DfaDefer d, int n_segs, MatchOut *out, int64_t cap) {
    for (int sg = blockIdx.x; sg < n_segs; sg += gridDim.x) {
        const long long at = d.seg_at[sg];
        if (at < 0) continue;
        const long long cnt = d.seg_cnt[sg], base = d.seg_base[sg];
        for (long long i = threadIdx.x; i < cnt; i += 256) {
            const long long o = base + i;
            if (o < cap) out[o] = d.stage[at + i];
        }
    }
}

template <int ENC>
const void *pick(bool id) {
    return id ? reinterpret_cast<const void *>(&dfa_scan_kernel<ENC, true>)
              : reinterpret_cast<const void *>(&dfa_scan_kernel<ENC, false>);
}

// Carried instances through a piece, one lane per instance reading the
// table, flags and labels through the cache hierarchy.  Count pass: matches
// per instance, and the instances still live after the piece go to the carry
// list; write pass: the matches, in (end, label) order, from the instance's
// output offset on.
__global__ __launch_bounds__(256) void dfa_resume_kernel(DfaResumeArgs r) {
    const int G = *r.in.n_groups;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
        const unsigned long long key = r.in.keys[r.in.grp_off[g]];
        const int32_t start = (int32_t)(key >> 32);
        int s = (int)(uint32_t)key;
        const long long at = r.write ? r.off[g] : 0;
        long long k = 0;
        bool alive = true;
        for (int64_t p = 0; p < r.n; ++p) {
            const int b = r.x[p];
            const int sy = r.identity ? b : (int)r.b2s[b];
            int t = -1;
            if (sy >= 0)
                t = r.tbl16 ? (int)reinterpret_cast<const int16_t *>(r.tbl)[(int64_t)s * r.n_symbols + sy]
                            : reinterpret_cast<const int32_t *>(r.tbl)[(int64_t)s * r.n_symbols + sy];
            if (t < 0 || !(r.flags[t] & kLive)) {
                alive = false;
                break;
            }
            s = t;
            const int lo = r.lab_off[s], hi = r.lab_off[s + 1];
            if (r.write) {
                for (int l = lo; l < hi; ++l, ++k)
                    if (at + k < r.cap) {
                        MatchOut *o = &r.out[at + k];
                        o->start = start;
                        o->end = r.base + (int32_t)p;
                        o->label = r.lab[l];
                    }
            } else {
                k += hi - lo;
            }
        }
        if (!r.write) {
            r.cnt[g] = k;
            if (alive) carry_write(r.carry, carry_reserve(r.carry, 1), start - r.carry.base, (uint32_t)s);
        }
    }
}

}  // namespace

hipError_t launch_dfa_resume(const DfaResumeArgs &r, hipStream_t s) {
    hipLaunchKernelGGL(dfa_resume_kernel, dim3(64), dim3(256), 0, s, r);
    return hipGetLastError();
}

const void *dfa_kernel_fn(int enc, bool identity_map) {
    switch (enc) {
    case kEnc8: return pick<kEnc8>(identity_map);
    case kEnc8D: return pick<kEnc8D>(identity_map);
    case kEnc16: return pick<kEnc16>(identity_map);
    case kCold16: return pick<kCold16>(identity_map);
    case kCold32: return pick<kCold32>(identity_map);
    default: return nullptr;
    }
}

hipError_t launch_dfa_place(const DfaDefer &d, int n_segs, int64_t *total, MatchOut *out, int64_t cap,
                            hipStream_t s) {
    if (n_segs <= kDeferFusedSegs) {
        dfa_place_fused_kernel<<<n_segs, 256, 0, s>>>(d, n_segs, total, out, cap);
        return hipGetLastError();
    }
    dfa_place_scan_kernel<<<1, 1024, 0, s>>>(d, n_segs, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = n_segs < 1 ? 1 : (n_segs < 2048 ? n_segs : 2048);
    dfa_place_copy_kernel<<<grid, 256, 0, s>>>(d, n_segs, out, cap);
    return hipGetLastError();
}

hipError_t launch_write_zero(int64_t *p, hipStream_t stream) {
    hipLaunchKernelGGL(write_zero_kernel, dim3(1), dim3(1), 0, stream, p);
    return hipGetLastError();
}

}  // namespace pfsmk
