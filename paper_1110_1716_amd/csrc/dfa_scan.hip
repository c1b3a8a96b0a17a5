// All-matches DFA scan for gfx950 (Section III.B with a deterministic
// transition function; Section III.C's DFA case).
//
// One workgroup owns the start positions of one window of W = 256*B bytes
// (lazy data partitioning, Section III.D.2: a window owns its starts and its
// walks read past its end until they die).  Per window:
//   1. stage x[base, base + W + kOverlap) from HBM into LDS, 16 B per load;
//   2. first step of every start (the tagged reinitialisation of q0 followed
//      by one symbol, Section III.B steps 1-4) from the q0 row cached in LDS,
//      indexed by byte;
//   3. survivors go to an LDS queue (ballot + prefix-sum compaction) and
//      advance kSteps symbols per round through the unmodified table (L2),
//      re-packed after every round, until the queue is empty;
//   4. every final state entered emits (start, end, label) into an LDS
//      buffer (Section III.B reporting rule);
//   5. the window's count goes through a decoupled look-back to get its
//      global offset; each buffered match is placed by its rank in
//      (start, end, label) order.  A window with more matches than the buffer
//      holds re-walks its starts 256 at a time, counting then writing.
#include "scan_common.h"

namespace pfsmk {

namespace {

constexpr int kQCap = 512;   // LDS queue entries per buffer (double-buffered)
constexpr int kMCap = 512;   // LDS match buffer entries
constexpr int kSteps = 4;    // symbols advanced per queue round

struct QEnt {
    int32_t start, state, pos, pad;
};
struct MEnt {
    int32_t start, end, label, pad;
};

template <typename TT, bool kId>
struct Dfa {
    const DfaArgs &a;
    const uint8_t *xs;
    const int32_t *first_s;
    const int16_t *b2s_s;
    const uint8_t *flags_s;
    int64_t base;
    int staged;
    bool flags_lds;

    __device__ __forceinline__ int byte_at(int32_t pos) const {
        const int64_t r = (int64_t)pos - base;
        return r < staged ? (int)xs[r] : (int)a.x[pos];
    }
    __device__ __forceinline__ uint8_t flag(int s) const { return flags_lds ? flags_s[s] : a.flags[s]; }
    // One symbol from state s: the target, or -1 when the instance ends.
    __device__ __forceinline__ int step(int s, int byte) const {
        const int sym = kId ? byte : (int)b2s_s[byte];
        if (sym < 0) return -1;
        const TT *t = reinterpret_cast<const TT *>(a.tbl);
        const int nx = (int)t[(int64_t)s * a.n_symbols + sym];
        if (nx < 0) return -1;
        return (flag(nx) & kLive) ? nx : -1;
    }
};

template <int B, typename TT, bool kId>
__global__ __launch_bounds__(kBlock) void dfa_scan_kernel(DfaArgs a) {
    constexpr int W = kBlock * B;
    constexpr int XS = W + kOverlap;
    __shared__ __align__(16) uint8_t xs[XS];
    __shared__ int32_t first_s[256];
    __shared__ int16_t b2s_s[256];
    __shared__ uint8_t flags_s[kFlagsLds];
    __shared__ QEnt q[2][kQCap];
    __shared__ MEnt mb[kMCap];
    __shared__ int qn[2];
    __shared__ int mn;
    __shared__ int ovf;
    __shared__ int last_flag;
    __shared__ unsigned wid_s;
    __shared__ long long red[kBlock / 64];
    __shared__ long long excl_s;

    const int tid = threadIdx.x;
    if (tid == 0) {
        wid_s = atomicAdd(&a.ctl->ticket, 1u);
        qn[0] = qn[1] = 0;
        mn = 0;
        ovf = 0;
    }
    first_s[tid] = a.first[tid];
    if (!kId) b2s_s[tid] = a.b2s[tid];
    const bool flags_lds = a.n_states <= kFlagsLds;
    if (flags_lds)
        for (int i = tid; i < a.n_states; i += kBlock) flags_s[i] = a.flags[i];
    __syncthreads();

    const long long w = wid_s;
    const int64_t base = w * (int64_t)W;
    const int64_t lim = a.n - base;  // starts owned: [base, base + min(W, lim))
    const int staged = (int)(lim < XS ? lim : XS);
    stage_bytes(xs, a.x + base, staged);
    __syncthreads();

    Dfa<TT, kId> d{a, xs, first_s, b2s_s, flags_s, base, staged, flags_lds};
    const int32_t n32 = (int32_t)a.n;
    long long tT = 0, tX = 0, tM = 0, tL = 0;

    auto emit = [&](int32_t start, int32_t end, int s) {
        const int lo = a.lab_off[s], hi = a.lab_off[s + 1];
        tM += hi - lo;
        for (int l = lo; l < hi; ++l) {
            if (ovf) break;
            const int slot = atomicAdd(&mn, 1);
            if (slot < kMCap) {
                mb[slot] = MEnt{start, end, a.lab[l], 0};
            } else {
                ovf = 1;
            }
        }
    };

    int cur = 0;
    // Advance every queued walk until the queue is empty.
    // Each round: every thread reads the count, a barrier guarantees that
    // before anyone pushes again, then survivors are re-packed into the other
    // buffer.
    auto drain = [&]() {
        for (;;) {
            __syncthreads();
            const int cnt = qn[cur];
            __syncthreads();
            if (cnt == 0) break;
            const int nxt = cur ^ 1;
            if (tid == 0) qn[cur] = 0;
            for (int e0 = 0; e0 < cnt; e0 += kBlock) {
                const int e = e0 + tid;
                bool alive = e < cnt;
                QEnt en{0, 0, 0, 0};
                if (alive) en = q[cur][e];
#pragma unroll 1
                for (int r = 0; r < kSteps && alive; ++r) {
                    if (en.pos >= n32) { alive = false; break; }
                    if ((int64_t)en.pos - base == staged) ++tL;
                    const int b = d.byte_at(en.pos);
                    ++tT;
                    const int s2 = d.step(en.state, b);
                    if (s2 < 0) { alive = false; break; }
                    ++tX;
                    if (d.flag(s2) & kFinal) emit(en.start, en.pos, s2);
                    en.state = s2;
                    ++en.pos;
                }
                if (alive && en.pos >= n32) alive = false;
                const int slot = wave_reserve(&qn[nxt], alive);
                if (alive) q[nxt][slot] = en;
            }
            cur = nxt;
        }
    };

    // First step of every start: q0 (tag = position) consumes its byte.
#pragma unroll 1
    for (int j = 0; j < B; ++j) {
        const int il = j * kBlock + tid;
        bool push = false;
        int s = -1;
        if (il < lim) {
            const int32_t i = (int32_t)(base + il);
            s = first_s[xs[il]];
            ++tT;
            if (s >= 0) {
                ++tX;
                if (d.flag(s) & kFinal) emit(i, i, s);
                push = i + 1 < n32;
            }
        }
        const int slot = wave_reserve(&qn[cur], push);
        if (push) q[cur][slot] = QEnt{(int32_t)(base + il), s, (int32_t)(base + il + 1), 0};
        __syncthreads();
        const int queued = qn[cur];
        __syncthreads();
        if (queued > kQCap - kBlock) drain();
    }
    drain();

    // Window total, look-back, placement.
    const long long wtot = block_sum(tM, red);
    if (tid < 64) {
        const long long ex = lookback(a.status, w, wtot);
        if (tid == 0) {
            excl_s = ex;
            if (w == a.n_windows - 1) *a.total = ex + wtot;
        }
    }
    __syncthreads();
    const long long excl = excl_s;

    if (!ovf) {
        const int m = mn;
        for (int e = tid; e < m; e += kBlock) {
            const MEnt me = mb[e];
            int rank = 0;
            for (int k = 0; k < m; ++k) {
                const MEnt o = mb[k];
                rank += (o.start < me.start) ||
                        (o.start == me.start && (o.end < me.end || (o.end == me.end && o.label < me.label)));
            }
            const long long at = excl + rank;
            if (at < a.cap) {
                MatchOut *p = &a.out[at];
                p->start = me.start;
                p->end = me.end;
                p->label = me.label;
            }
        }
    } else {
        // Dense window: 256 starts at a time, thread order = start order.
        long long run = excl;
#pragma unroll 1
        for (int c = 0; c < B; ++c) {
            const int il = c * kBlock + tid;
            const bool own = il < lim;
            const int32_t i = (int32_t)(base + il);
            long long cnt = 0;
            if (own) {
                int s = first_s[xs[il]];
                int32_t pos = i;
                while (s >= 0) {
                    cnt += a.lab_off[s + 1] - a.lab_off[s];
                    if (++pos >= n32) break;
                    s = d.step(s, d.byte_at(pos));
                }
            }
            long long ctot;
            const long long ex = block_excl_scan(cnt, red, &ctot);
            if (own && cnt) {
                long long at = run + ex;
                int s = first_s[xs[il]];
                int32_t pos = i;
                while (s >= 0) {
                    for (int l = a.lab_off[s]; l < a.lab_off[s + 1]; ++l, ++at) {
                        if (at < a.cap) {
                            MatchOut *p = &a.out[at];
                            p->start = i;
                            p->end = pos;
                            p->label = a.lab[l];
                        }
                    }
                    if (++pos >= n32) break;
                    s = d.step(s, d.byte_at(pos));
                }
            }
            run += ctot;
        }
    }

    const long long bT = block_sum(tT, red);
    const long long bX = block_sum(tX, red);
    const long long bL = block_sum(tL, red);
    finish_launch(a.ctl, a.status, a.n_windows, bT, bX, bL, wtot, &last_flag);
}

__global__ void write_zero_kernel(int64_t *p) { *p = 0; }

template <int B, typename TT, bool kId>
hipError_t launch_one(const DfaArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((dfa_scan_kernel<B, TT, kId>), dim3(a.n_windows), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int B>
hipError_t launch_b(const DfaArgs &a, bool id, bool t16, hipStream_t s) {
    if (t16) return id ? launch_one<B, int16_t, true>(a, s) : launch_one<B, int16_t, false>(a, s);
    return id ? launch_one<B, int32_t, true>(a, s) : launch_one<B, int32_t, false>(a, s);
}

}  // namespace

hipError_t launch_dfa_scan(const DfaArgs &a, int per_thread, bool identity_map, bool tbl16,
                           hipStream_t stream) {
    switch (per_thread) {
    case 1: return launch_b<1>(a, identity_map, tbl16, stream);
    case 4: return launch_b<4>(a, identity_map, tbl16, stream);
    case 16: return launch_b<16>(a, identity_map, tbl16, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_write_zero(int64_t *p, hipStream_t stream) {
    hipLaunchKernelGGL(write_zero_kernel, dim3(1), dim3(1), 0, stream, p);
    return hipGetLastError();
}

}  // namespace pfsmk
