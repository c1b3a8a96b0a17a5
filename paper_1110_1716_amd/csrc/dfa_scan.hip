// All-matches DFA scan for gfx950 (Section III.B with a deterministic
// transition function; the DFA case of Section III.C).
//
// Persistent cooperative grid of 768-thread workgroups (12 wave64, one per
// compute unit when the table is resident in LDS).  Workgroup b owns the
// start positions of one contiguous segment per round (lazy data
// partitioning, Section III.D.2: a segment owns its starts, its walks read
// past its end until they die).  The segment is processed in windows of 16 bytes per thread:
//   1. the window (12 KiB) is staged from HBM into LDS with 16-byte loads issued two
//      windows ahead;
//   2. every start takes its first symbol through the row of q0 cached in LDS
//      by byte (Section III.B steps 1-4 for the fresh tag), 16 independent
//      lookups per thread; the live ones take their second symbol through
//      the table (resident in LDS, or the LDS copies of q0's successor rows);
//   3. walks still live go to a wave-private LDS queue (ballot + prefix
//      popcount) and advance in rounds of up to 16 symbols per walk, the
//      symbols coming from one 16-byte chunk (LDS inside the window, L2
//      outside it); walks left at the end of a window carry over;
//   4. every final state entered adds (start, end, label) to an LDS buffer
//      under the key (start - segment start, k), k = the instance's match
//      count so far, which orders (end, label) within a start (Section III.B
//      reporting rule).
// At the end of a round each workgroup publishes its match count in its own
// epoch-tagged slot and sums its peers' slots (no shared counters), then
// writes every buffered match at its rank.  A segment whose matches do not
// fit the buffer is re-walked 768 starts at a time: count, scan, write.
#include "scan_common.h"

namespace pfsmk {

namespace {

constexpr int NT = kDfaThreads;
constexpr int W = kDfaWindow;
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
    const int32_t *first_s;
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
    int64_t wbase;
    int staged;
    int64_t seg_lo;
    int32_t n32;
    long long T = 0, X = 0, L = 0, M = 0;

    static constexpr bool kResident = ENC == kEnc8 || ENC == kEnc8D || ENC == kEnc16;

    __device__ __forceinline__ uint8_t flag(int s) const {
        if constexpr (kResident) return flags_s[s];
        else return a.flags[s];
    }
    __device__ __forceinline__ int sym(int byte) const { return kId ? byte : (int)b2s_s[byte]; }
    // delta(s, sy) as given: a state or -1.
    __device__ __forceinline__ int tab(int s, int sy) const {
        const int64_t i = (int64_t)s * a.n_symbols + sy;
        if constexpr (ENC == kEnc8) {
            const int v = tab_s[i];
            return v == 255 ? -1 : v;
        } else if constexpr (ENC == kEnc8D) {
            const int ns = a.n_states * a.n_symbols;
            const uint32_t *dead = reinterpret_cast<const uint32_t *>(tab_s + ((ns + 3) & ~3));
            return (dead[i >> 5] >> (i & 31)) & 1u ? -1 : (int)tab_s[i];
        } else if constexpr (ENC == kEnc16) {
            return reinterpret_cast<const int16_t *>(tab_s)[i];
        } else if constexpr (ENC == kCold16) {
            return reinterpret_cast<const int16_t *>(a.tbl)[i];
        } else {
            return reinterpret_cast<const int32_t *>(a.tbl)[i];
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
                    mend[slot + l] = end;
                    mlab[slot + l] = lab_at(lo + l);
                }
            } else {
                *ovf = 1;
            }
        }
        k += cnt;
    }
    __device__ __forceinline__ int n_labels(int s) const { return lab_lo(s + 1) - lab_lo(s); }
    // The 16-byte chunk holding position p (p is a multiple of 16).
    __device__ __forceinline__ uint4 chunk(int64_t p) {
        const int64_t r = p - wbase;
        if (r >= 0 && r + 16 <= staged) return *reinterpret_cast<const uint4 *>(xs + r);
        ++L;
        return load_granule(a.x, p);
    }
};

// One round: every walk in this wave's queue advances through the rest of
// the 16-byte chunk holding its next position (up to 16 symbols); walks that
// end are dropped and the queue is re-packed.
template <int ENC, bool kId>
__device__ __forceinline__ void drain_round(DfaCtx<ENC, kId> &c, QEnt *q, int &qcount) {
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
        ch[j] = alive[j] ? c.chunk(c0) : make_uint4(0, 0, 0, 0);
        const int64_t end = c0 + 16 < c.a.n ? c0 + 16 : c.a.n;
        steps[j] = (int)(end - e[j].pos);  // symbols left in this chunk
    }
    // t[j]: target of the walk's next symbol, looked up one step ahead so
    // that the flag read of a state overlaps the table read of its successor.
    int t[QK];
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const int sy = c.sym(byte_of(ch[j], e[j].pos & 15));
        t[j] = (alive[j] && sy >= 0) ? c.tab(e[j].state, sy) : -1;
    }
#pragma unroll 1
    for (int st = 0; st < 16; ++st) {
        bool more = false;
#pragma unroll
        for (int j = 0; j < QK; ++j) {
            if (alive[j] && st < steps[j]) {
                ++c.T;
                const int cur = t[j];
                if (cur < 0) {
                    alive[j] = false;
                } else {
                    const uint8_t f = c.flag(cur);
                    int nxt = -1;
                    if (st + 1 < steps[j]) {
                        const int sy = c.sym(byte_of(ch[j], (e[j].pos + 1) & 15));
                        if (sy >= 0) nxt = c.tab(cur, sy);
                    }
                    if (!(f & kLive)) {
                        alive[j] = false;
                    } else {
                        ++c.X;
                        if (f & kFinal) c.emit(e[j].start, e[j].pos, cur, e[j].k);
                        e[j].state = cur;
                        ++e[j].pos;
                        t[j] = nxt;
                        more |= st + 1 < steps[j];
                    }
                }
            }
        }
        if (!__any(more)) break;
    }
    int nc = 0;
#pragma unroll
    for (int j = 0; j < QK; ++j) {
        const bool keep = alive[j] && e[j].pos < c.n32;
        const int slot = wave_push_slot(nc, keep);
        if (keep) q[slot] = e[j];
    }
    __builtin_amdgcn_wave_barrier();
    qcount = nc;
}

// The full walk of one start reading the input through the cache hierarchy;
// counts its matches, or writes them from output index `at` when write.
template <int ENC, bool kId>
__device__ __forceinline__ long long walk_start(const DfaCtx<ENC, kId> &c, int32_t i, bool write, long long at) {
    const DfaArgs &a = c.a;
    long long cnt = 0;
    int s = c.first_s[a.x[i]];
    int32_t pos = i;
    while (s >= 0) {
        for (int l = c.lab_lo(s); l < c.lab_lo(s + 1); ++l, ++cnt) {
            if (write && at + cnt < a.cap) {
                MatchOut *p = &a.out[at + cnt];
                p->start = i;
                p->end = pos;
                p->label = c.lab_at(l);
            }
        }
        if (++pos >= c.n32) break;
        const int sy = c.sym(a.x[pos]);
        s = sy < 0 ? -1 : c.live(c.tab(s, sy));
    }
    return cnt;
}

template <int ENC, bool kId>
__global__ __launch_bounds__(NT) void dfa_scan_kernel(DfaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *xs = lds;
    int32_t *first_s = reinterpret_cast<int32_t *>(lds + W);
    int16_t *slot_s = reinterpret_cast<int16_t *>(first_s + 256);
    int16_t *b2s_s = slot_s + 256;
    uint8_t *flags_s = lds + a.off_flags;
    int32_t *laboff_s = reinterpret_cast<int32_t *>(lds + a.off_laboff);
    int32_t *lab_s = reinterpret_cast<int32_t *>(lds + a.off_lab);
    uint8_t *tab_s = lds + a.off_tab;
    QEnt *qall = reinterpret_cast<QEnt *>(lds + a.off_q);
    uint32_t *mkey = reinterpret_cast<uint32_t *>(lds + a.off_m);
    uint16_t *list_all = reinterpret_cast<uint16_t *>(lds + a.off_list);
    int32_t *mend = reinterpret_cast<int32_t *>(mkey + MC);
    int32_t *mlab = mend + MC;
    __shared__ int mn, ovf;
    __shared__ long long red[NT / 64];
    __shared__ long long red4[4 * (NT / 64)];
    __shared__ unsigned epoch_s;

    const int tid = threadIdx.x;
    const int wv = tid >> 6;
    const int b = blockIdx.x;
    const int32_t n32 = (int32_t)a.n;

    // Issue the first two windows' loads before anything else.
    auto seg_of = [&](int r, int64_t &lo, int64_t &hi) __attribute__((always_inline)) {
        lo = ((int64_t)r * a.n_blocks + b) * a.seg;
        hi = lo + a.seg < a.n ? lo + a.seg : a.n;
    };
    int64_t seg_lo, seg_hi;
    seg_of(0, seg_lo, seg_hi);
    // Window stream over the rounds: (round, window base) in order.
    int pr = 0;
    int64_t pw = seg_lo, plo = seg_lo, phi = seg_hi;
    auto next_window = [&](int64_t &wb, bool &ok) __attribute__((always_inline)) {
        // advance (pr, pw) to the next window that has starts
        while (pr < a.n_rounds) {
            if (pw < phi) {
                wb = pw;
                pw += W;
                ok = true;
                return;
            }
            ++pr;
            if (pr < a.n_rounds) {
                seg_of(pr, plo, phi);
                pw = plo;
            }
        }
        ok = false;
    };
    auto fetch = [&](int64_t wb, uint4 &v) __attribute__((always_inline)) {
        const int64_t p = wb + 16 * tid;
        v = p < a.n ? load_granule(a.x, p) : make_uint4(0, 0, 0, 0);
    };
    // Two prefetch buffers used alternately: buffer p holds the window
    // after next while the other one's window is being processed.
    int64_t pwb[2] = {0, 0};
    bool pok[2] = {false, false};
    uint4 pv[2];
    next_window(pwb[0], pok[0]);
    if (pok[0]) fetch(pwb[0], pv[0]);
    next_window(pwb[1], pok[1]);
    if (pok[1]) fetch(pwb[1], pv[1]);

    // Tables into LDS.
    if (tid < 256) {
        first_s[tid] = a.first[tid];
        slot_s[tid] = a.first_slot[tid];
        b2s_s[tid] = a.b2s[tid];
    }
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.res);
        uint4 *dst = reinterpret_cast<uint4 *>(tab_s);
        for (int i = tid; i < (a.res_bytes >> 4); i += NT) dst[i] = src[i];
    }
    if (DfaCtx<ENC, kId>::kResident) {
        for (int i = tid; i < a.n_states; i += NT) flags_s[i] = a.flags[i];
        for (int i = tid; i <= a.n_states; i += NT) laboff_s[i] = a.lab_off[i];
        const int nnz = a.lab_off[a.n_states];
        for (int i = tid; i < nnz; i += NT) lab_s[i] = a.lab[i];
    }
    if (tid == 0) {
        mn = 0;
        ovf = 0;
        epoch_s = first_epoch(a.slots, b);
    }
    __syncthreads();
    const unsigned epoch0 = epoch_s;

    DfaCtx<ENC, kId> c{a, xs, first_s, slot_s, b2s_s, flags_s, laboff_s, lab_s, tab_s, mkey,
                       mend, mlab, &mn, &ovf, 0, 0, 0, n32};
    QEnt *q = qall + wv * QW;
    int qcount = 0;
    long long base_out = 0;

    // Process the window held in prefetch buffer p, then refill p with the
    // window two ahead.  Called with p = 0, 1, 0, 1, ... (static indices).
    auto run_window = [&](const int p) __attribute__((always_inline)) {
        const int64_t wbase = pwb[p];
        const int64_t wend = wbase + W < seg_hi ? wbase + W : seg_hi;
        const int64_t rest = a.n - wbase;
        const int staged = (int)(rest < W ? rest : W);
        __syncthreads();  // every wave is done with the previous window's bytes
        *reinterpret_cast<uint4 *>(xs + 16 * tid) = pv[p];
        const uint4 mine = pv[p];
        next_window(pwb[p], pok[p]);
        if (pok[p]) fetch(pwb[p], pv[p]);
        __syncthreads();
        c.wbase = wbase;
        c.staged = staged;

        // Symbol one for the 16 starts owned by this thread: 16 independent
        // lookups of the q0 row, giving the mask of live instances.
        const int il0 = 16 * tid;
        const int64_t i0 = wbase + il0;
        const int64_t nv64 = wend - i0;
        const int nvalid = nv64 <= 0 ? 0 : (nv64 >= 16 ? 16 : (int)nv64);
        unsigned lm = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < nvalid && first_s[byte_of(mine, k)] >= 0) lm |= 1u << k;
        c.T += nvalid;
        c.X += __popc(lm);
        // Compact the wave's live instances into its LDS list (prefix sum of
        // the lanes' counts), then advance them with every lane busy.
        const int cnt = __popc(lm);
        const int incl = (int)wave_incl_scan(cnt);
        const int total = __shfl(incl, 63);
        int off = incl - cnt;
        uint16_t *lst = list_all + wv * (64 * 16);
        while (lm) {
            const int k = __ffs(lm) - 1;
            lm &= lm - 1;
            lst[off++] = (uint16_t)(il0 + k);
        }
        __builtin_amdgcn_wave_barrier();
        for (int e0 = 0; e0 < total; e0 += 64) {
            const int e = e0 + lane_id();
            bool push = false;
            QEnt ent{0, 0, 0, 0};
            if (e < total) {
                const int il = lst[e];
                const int32_t i = (int32_t)(wbase + il);
                const int b0 = xs[il];
                const int s1 = first_s[b0];
                int32_t km = 0;
                if (c.flag(s1) & kFinal) c.emit(i, i, s1, km);
                if (i + 1 < n32) {
                    ++c.T;
                    const int b1 = il + 1 < staged ? xs[il + 1] : a.x[i + 1];
                    const int sy = c.sym(b1);
                    const int t2 = sy < 0 ? -1 : c.live(c.tab2(b0, s1, sy));
                    if (t2 >= 0) {
                        ++c.X;
                        if (c.flag(t2) & kFinal) c.emit(i, i + 1, t2, km);
                        if (i + 2 < n32) {
                            push = true;
                            ent = QEnt{i, t2, i + 2, km};
                        }
                    }
                }
            }
            while (qcount > QW - 64) drain_round(c, q, qcount);
            const int slot = wave_push_slot(qcount, push);
            if (push) q[slot] = ent;
        }
    };

    for (int r = 0; r < a.n_rounds; ++r) {
        seg_of(r, seg_lo, seg_hi);
        c.seg_lo = seg_lo;
        const long long m_before = c.M;
        auto in_round = [&](int p) __attribute__((always_inline)) { return pok[p] && pwb[p] >= seg_lo && pwb[p] < seg_hi; };
        for (;;) {
            if (!in_round(0)) break;
            run_window(0);
            if (!in_round(1)) break;
            run_window(1);
        }
        // The round's walks run to their end.
        while (qcount > 0) drain_round(c, q, qcount);

        // Offsets: this round's count, the peers' counts, placement.
        const long long mine_m = block_sum<NT>(c.M - m_before, red);
        long long round_total;
        const long long excl =
            grid_prefix<NT>(a.slots, a.n_blocks, b, (epoch0 + r) & kEpochMask, mine_m, red, &round_total);
        const long long at0 = base_out + excl;
        if (!ovf) {
            // Rank of every buffered match in (start, end, label) order:
            // bucket by start offset / 64 (histogram, scan, scatter), then
            // compare within the bucket.  The queue area is free here.
            const int m = mn;
            int *hist = reinterpret_cast<int *>(qall);
            int *base = hist + 1024;
            int *fill = base + 1024;
            int *memb = fill + 1024;
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
                const int bk = mkey[e] >> 22;
                memb[base[bk] + atomicAdd(&fill[bk], 1)] = e;
            }
            __syncthreads();
            for (int e = tid; e < m; e += NT) {
                const uint32_t mk = mkey[e];
                const int bk = mk >> 22;
                int rank = base[bk];
                for (int j = base[bk]; j < base[bk] + hist[bk]; ++j) rank += mkey[memb[j]] < mk;
                const long long at = at0 + rank;
                if (at < a.cap) {
                    MatchOut *p = &a.out[at];
                    p->start = (int32_t)(seg_lo + (mk >> 16));
                    p->end = mend[e];
                    p->label = mlab[e];
                }
            }
        } else {
            long long run = at0;
            for (int64_t c0 = seg_lo; c0 < seg_hi; c0 += NT) {
                const int64_t i = c0 + tid;
                const bool own = i < seg_hi;
                const long long cnt = own ? walk_start(c, (int32_t)i, false, 0) : 0;
                long long ctot;
                const long long ex = block_excl_scan<NT>(cnt, red, &ctot);
                if (own && cnt) walk_start(c, (int32_t)i, true, run + ex);
                run += ctot;
            }
        }
        base_out += round_total;
        __syncthreads();
        if (tid == 0) {
            mn = 0;
            ovf = 0;
        }
    }
    if (b == 0 && tid == 0) *a.total = base_out;
    long long st4[4] = {c.T, c.X, c.L, c.M};
    block_sum4<NT>(st4, red4);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.bstats[4 * b + k] = st4[k];
    }
}

__global__ void write_zero_kernel(int64_t *p) { *p = 0; }

template <int ENC>
const void *pick(bool id) {
    return id ? reinterpret_cast<const void *>(&dfa_scan_kernel<ENC, true>)
              : reinterpret_cast<const void *>(&dfa_scan_kernel<ENC, false>);
}

}  // namespace

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

hipError_t launch_write_zero(int64_t *p, hipStream_t stream) {
    hipLaunchKernelGGL(write_zero_kernel, dim3(1), dim3(1), 0, stream, p);
    return hipGetLastError();
}

}  // namespace pfsmk
