// Streaming scans: a stream's bytes arrive in pieces, and the matches of the
// pieces together are those of one scan of the whole stream.  This is the
// chained form of data partitioning (Section III.D.2): an instance still
// live when a piece ends is handed to the next piece as (start, state set)
// and continues there, so no piece re-reads earlier bytes.
//
// A piece of n bytes at stream position base runs, on one HIP stream:
//   1. resume, count pass: each carried instance advances through the piece;
//      its match count, and (if it is still live after the piece) its state
//      set as carry pairs;
//   2. an exclusive scan of those counts: R, the matches of carried
//      instances, all of which precede the piece's own (smaller starts);
//   3. the ordinary scan of the piece with its output placed from R on and
//      its instances live at the end appended as carry pairs;
//   4. resume, write pass: the carried instances' matches into [0, R);
//   5. positions of the piece's own matches moved from piece to stream
//      coordinates;
//   6. after one synchronisation (the match total and the pair count): the
//      carry pairs become sorted unique keys grouped by start, the carried
//      set of the next piece (one workgroup sorts a few thousand pairs in
//      LDS; more are sorted in LDS tiles of 2048 keys, then merged pairwise
//      in passes over device memory).
// The stream state changes only when a piece succeeds, so a piece refused
// for lack of output room can be fed again with a larger buffer.
#include <algorithm>
#include <cstring>
#include <new>
#include <utility>

#include "host_common.h"
#include "pfsm.h"
#include "pfsm_dev.h"
#include "scan_common.h"
#include "stream.h"

struct pfsm;

namespace pfsmk {

uint64_t handle_edits(const pfsm *h);
int piece_scan(pfsm *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap, int64_t *d_total,
               const int64_t *d_base, const CarryOut *carry, hipStream_t s);
int piece_resume(pfsm *h, const uint8_t *x, int64_t n, int32_t base, const CarrySet &in, int64_t *cnt,
                 const int64_t *off, MatchOut *out, int64_t cap, const CarryOut &carry, int write, hipStream_t s);

namespace {

constexpr int ST = 1024;

__global__ void zero2_kernel(unsigned long long *a, int64_t *b) {
    *a = 0;
    *b = 0;
}

// Exclusive scan of the per-instance match counts; *total = their sum.
__global__ __launch_bounds__(ST) void count_scan_kernel(const int64_t *cnt, const int32_t *n_groups, int64_t *off,
                                                        int64_t *total) {
    __shared__ long long red[ST / 64];
    const int G = *n_groups;
    long long run = 0;
    for (int c0 = 0; c0 < G; c0 += ST) {
        const int g = c0 + threadIdx.x;
        long long tot;
        const long long ex = block_excl_scan<ST>(g < G ? cnt[g] : 0, red, &tot);
        if (g < G) off[g] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) *total = run;
}

// Piece positions of out[*lo, min(*hi, cap)) to stream positions.
__global__ void shift_kernel(MatchOut *out, const int64_t *lo, const int64_t *hi, int64_t cap, int32_t base) {
    const int64_t a = *lo, b = *hi < cap ? *hi : cap;
    for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += (int64_t)gridDim.x * blockDim.x) {
        out[i].start += base;
        out[i].end += base;
    }
}

// Sorted keys to unique keys and the offsets of their start groups.
__global__ __launch_bounds__(ST) void compact_kernel(const unsigned long long *sorted, int64_t m,
                                                     unsigned long long *keys, int32_t *grp_off, int32_t *n_groups) {
    __shared__ long long red[ST / 64];
    long long run_u = 0, run_g = 0;
    for (int64_t c0 = 0; c0 < m; c0 += ST) {
        const int64_t i = c0 + threadIdx.x;
        const bool in = i < m;
        const unsigned long long k = in ? sorted[i] : 0;
        const unsigned long long prev = in && i > 0 ? sorted[i - 1] : 0;
        const bool uniq = in && (i == 0 || k != prev);
        const bool head = in && (i == 0 || (k >> 32) != (prev >> 32));
        long long tot_u, tot_g;
        const long long ex_u = block_excl_scan<ST>(uniq ? 1 : 0, red, &tot_u);
        const long long ex_g = block_excl_scan<ST>(head ? 1 : 0, red, &tot_g);
        if (uniq) keys[run_u + ex_u] = k;
        if (head) grp_off[run_g + ex_g] = (int32_t)(run_u + ex_u);
        run_u += tot_u;
        run_g += tot_g;
    }
    if (threadIdx.x == 0) {
        grp_off[run_g] = (int32_t)run_u;
        *n_groups = (int32_t)run_g;
    }
}

__device__ __forceinline__ unsigned long long pair_key(const uint32_t *pairs, int64_t i) {
    return ((unsigned long long)pairs[2 * i] << 32) | pairs[2 * i + 1];
}

// Bitonic sort of np keys in LDS (np a power of two, at most 2048), by the
// whole workgroup.  Keys are below 2^63 (starts below 2^31), so the ~0
// padding sorts last.
__device__ __forceinline__ void bitonic_lds(unsigned long long *k_s, int np) {
    const int tid = threadIdx.x;
    for (int size = 2; size <= np; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < np; i += ST) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = k_s[i], b = k_s[j];
                    if ((a > b) == up) {
                        k_s[i] = b;
                        k_s[j] = a;
                    }
                }
            }
            __syncthreads();
        }
}

// Sort, deduplicate and group at most kSmallCarry pairs in one workgroup
// (bitonic sort of the keys in LDS), for the usual case of a few carried
// instances: one launch.
constexpr int kSmallCarry = 2048;

__global__ __launch_bounds__(ST) void small_carry_kernel(const uint32_t *pairs, int m, unsigned long long *keys,
                                                         int32_t *grp_off, int32_t *n_groups) {
    __shared__ unsigned long long k_s[kSmallCarry];
    __shared__ long long red[ST / 64];
    const int tid = threadIdx.x;
    int np = 1;
    while (np < m) np <<= 1;
    for (int i = tid; i < np; i += ST) k_s[i] = i < m ? pair_key(pairs, i) : ~0ull;
    __syncthreads();
    bitonic_lds(k_s, np);
    long long run_u = 0, run_g = 0;
    for (int c0 = 0; c0 < m; c0 += ST) {
        const int i = c0 + tid;
        const bool in = i < m;
        const unsigned long long k = in ? k_s[i] : 0;
        const unsigned long long prev = in && i > 0 ? k_s[i - 1] : 0;
        const bool uniq = in && (i == 0 || k != prev);
        const bool head = in && (i == 0 || (k >> 32) != (prev >> 32));
        long long tot_u, tot_g;
        const long long ex_u = block_excl_scan<ST>(uniq ? 1 : 0, red, &tot_u);
        const long long ex_g = block_excl_scan<ST>(head ? 1 : 0, red, &tot_g);
        if (uniq) keys[run_u + ex_u] = k;
        if (head) grp_off[run_g + ex_g] = (int32_t)(run_u + ex_u);
        run_u += tot_u;
        run_g += tot_g;
    }
    if (tid == 0) {
        grp_off[run_g] = (int32_t)run_u;
        *n_groups = (int32_t)run_g;
    }
}

// More carry pairs: each workgroup sorts one tile of kSmallCarry keys in
// LDS and writes its valid keys back in order.
__global__ __launch_bounds__(ST) void tile_sort_kernel(const uint32_t *pairs, int64_t m, unsigned long long *dst) {
    __shared__ unsigned long long k_s[kSmallCarry];
    const int64_t t0 = (int64_t)blockIdx.x * kSmallCarry;
    const int cnt = m - t0 < kSmallCarry ? (int)(m - t0) : kSmallCarry;
    for (int i = threadIdx.x; i < kSmallCarry; i += ST) k_s[i] = i < cnt ? pair_key(pairs, t0 + i) : ~0ull;
    __syncthreads();
    bitonic_lds(k_s, kSmallCarry);
    for (int i = threadIdx.x; i < cnt; i += ST) dst[t0 + i] = k_s[i];
}

// One merge pass: sorted runs of `width` keys (the last one shorter) are
// merged in pairs.  A key's place in the merged run is its index in its own
// run plus the number of keys of the other run that precede it, found by
// binary search; on equal keys the left run's come first.  Every key moves
// on its own, so the pass needs no synchronisation.
__global__ __launch_bounds__(256) void merge_pass_kernel(const unsigned long long *src, unsigned long long *dst,
                                                         int64_t m, int64_t width) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = i / (2 * width) * (2 * width);
        const int64_t mid = lo + width < m ? lo + width : m;
        const int64_t end = lo + 2 * width < m ? lo + 2 * width : m;
        const unsigned long long k = src[i];
        int64_t a, b;
        if (i < mid) {  // left run: right keys strictly smaller
            a = mid;
            b = end;
            while (a < b) {
                const int64_t h = (a + b) >> 1;
                if (src[h] < k) a = h + 1;
                else b = h;
            }
            dst[i + (a - mid)] = k;
        } else {  // right run: left keys smaller or equal
            a = lo;
            b = mid;
            while (a < b) {
                const int64_t h = (a + b) >> 1;
                if (src[h] <= k) a = h + 1;
                else b = h;
            }
            dst[lo + (i - mid) + (a - lo)] = k;
        }
    }
}

template <typename T>
int grow_dev(T **p, int64_t *cap, int64_t need, hipStream_t s) {
    if (need <= *cap) return PFSM_OK;
    HIP_TRY(hipStreamSynchronize(s));
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    const int64_t want = need + need / 2 + 256;
    HIP_TRY(hipMalloc(p, sizeof(T) * (size_t)want));
    *cap = want;
    return PFSM_OK;
}

}  // namespace
}  // namespace pfsmk

using namespace pfsmk;

struct pfsm_stream {
    pfsm *h = nullptr;
    uint64_t edits = 0;
    int device = 0;
    int64_t position = 0;  // stream position of the next piece
    // carried set: two copies, `cur` in use, the other built by a piece
    unsigned long long *keys[2] = {nullptr, nullptr};
    int64_t c_keys[2] = {0, 0};
    int32_t *grp[2] = {nullptr, nullptr};
    int64_t c_grp[2] = {0, 0};
    int32_t *n_groups = nullptr;  // [2]
    int cur = 0;
    int64_t bound = 0;  // at most this many carried instances (pairs before compaction)
    // per-piece buffers
    uint32_t *pairs = nullptr;
    int64_t c_pairs = 0;
    int64_t *d_back = nullptr;  // [2]: match total, carry pairs asked for (read back together)
    unsigned long long *sort_in = nullptr, *sort_out = nullptr;  // merge passes alternate between them
    int64_t c_sort_in = 0, c_sort_out = 0;
    int64_t *cnt = nullptr, *off = nullptr;
    int64_t c_cnt = 0, c_off = 0;
    int64_t *d_r = nullptr;
    int64_t *h_back = nullptr;  // pinned mirror of d_back

    ~pfsm_stream() {
        for (int i = 0; i < 2; ++i) {
            if (keys[i]) (void)hipFree(keys[i]);
            if (grp[i]) (void)hipFree(grp[i]);
        }
        void *dev[] = {n_groups, pairs, d_back, sort_in, sort_out, cnt, off, d_r};
        for (void *p : dev)
            if (p) (void)hipFree(p);
        if (h_back) (void)hipHostFree(h_back);
    }
};

extern "C" {

int pfsm_stream_open(pfsm_stream_t **out, pfsm_t *h) {
    if (!out || !h) return fail(PFSM_EINVAL, "NULL argument");
    *out = nullptr;
    pfsm_stream *st = new (std::nothrow) pfsm_stream;
    if (!st) return fail(PFSM_ENOMEM, "stream");
    st->h = h;
    st->edits = handle_edits(h);
    int rc = PFSM_OK;
    auto bad = [&](hipError_t e) {
        if (e != hipSuccess) rc = fail(PFSM_EHIP, "%s", hipGetErrorString(e));
        return e != hipSuccess;
    };
    if (bad(hipGetDevice(&st->device)) || bad(hipMalloc(&st->n_groups, 2 * sizeof(int32_t))) ||
        bad(hipMemset(st->n_groups, 0, 2 * sizeof(int32_t))) || bad(hipMalloc(&st->d_back, 2 * sizeof(int64_t))) ||
        bad(hipMalloc(&st->d_r, sizeof(int64_t))) ||
        bad(hipHostMalloc(&st->h_back, 2 * sizeof(int64_t), hipHostMallocDefault)) ||
        bad(hipDeviceSynchronize())) {
        delete st;
        return rc;
    }
    *out = st;
    return PFSM_OK;
}

int pfsm_stream_feed(pfsm_stream_t *st, const uint8_t *d_piece, int64_t n, pfsm_match_t *d_out, int64_t cap,
                     int64_t *n_matches, void *hip_stream) {
    if (!st || !n_matches) return fail(PFSM_EINVAL, "NULL argument");
    if (n < 0 || cap < 0) return fail(PFSM_EINVAL, "n and cap must be >= 0");
    if (n > 0 && !d_piece) return fail(PFSM_EINVAL, "d_piece is NULL");
    if (cap > 0 && !d_out) return fail(PFSM_EINVAL, "d_out is NULL");
    if (handle_edits(st->h) != st->edits)
        return fail(PFSM_EINVAL, "the automaton was edited after the stream was opened");
    *n_matches = 0;
    if (n == 0) return PFSM_OK;  // no symbol consumed: the carried set stays as it is
    if (n > kMaxStream - st->position)
        return fail(PFSM_EINVAL, "stream positions must stay below 2^31 - 16 (at %lld, piece of %lld)",
                    (long long)st->position, (long long)n);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != st->device) return fail(PFSM_EINVAL, "stream opened on device %d, current device %d", st->device, dev);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    MatchOut *out = reinterpret_cast<MatchOut *>(d_out);
    const int32_t base = (int32_t)st->position;
    const int cur = st->cur;
    const CarrySet in{st->keys[cur], st->grp[cur], st->n_groups + cur};
    int rc;
    if ((rc = grow_dev(&st->cnt, &st->c_cnt, st->bound, s)) || (rc = grow_dev(&st->off, &st->c_off, st->bound, s)) ||
        (rc = grow_dev(&st->pairs, &st->c_pairs, 1024, s)))
        return rc;
    for (;;) {
        unsigned long long *n_pairs = reinterpret_cast<unsigned long long *>(st->d_back + 1);
        const CarryOut co{st->pairs, n_pairs, st->c_pairs / 2, base, 0};
        hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(1), 0, s, n_pairs, st->d_r);
        HIP_TRY(hipGetLastError());
        if (st->bound > 0) {
            if ((rc = piece_resume(st->h, d_piece, n, base, in, st->cnt, nullptr, nullptr, 0, co, 0, s))) return rc;
            hipLaunchKernelGGL(count_scan_kernel, dim3(1), dim3(ST), 0, s, st->cnt, in.n_groups, st->off, st->d_r);
            HIP_TRY(hipGetLastError());
        }
        if ((rc = piece_scan(st->h, d_piece, n, out, cap, st->d_back, st->d_r, &co, s))) return rc;
        if (st->bound > 0 && cap > 0)
            if ((rc = piece_resume(st->h, d_piece, n, base, in, nullptr, st->off, out, cap, co, 1, s))) return rc;
        if (cap > 0) {
            hipLaunchKernelGGL(shift_kernel, dim3(256), dim3(256), 0, s, out, st->d_r, st->d_back, cap, base);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipMemcpyAsync(st->h_back, st->d_back, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int64_t want = st->h_back[1];
        if (want <= st->c_pairs / 2) break;
        // more carry pairs than room: grow and run the piece again
        if ((rc = grow_dev(&st->pairs, &st->c_pairs, 2 * want, s))) return rc;
    }
    const int64_t total = st->h_back[0];
    const int64_t m = st->h_back[1];
    if (m >= (int64_t)INT32_MAX) return fail(PFSM_ENOMEM, "%lld carried states", (long long)m);
    *n_matches = total;
    if (total > cap)
        return fail(PFSM_EOVERFLOW, "%lld matches, capacity %lld", (long long)total, (long long)cap);
    // The pairs become the next piece's carried set.
    const int nx = 1 - cur;
    if ((rc = grow_dev(&st->keys[nx], &st->c_keys[nx], m, s)) ||
        (rc = grow_dev(&st->grp[nx], &st->c_grp[nx], m + 1, s)))
        return rc;
    if (m > kSmallCarry &&
        ((rc = grow_dev(&st->sort_in, &st->c_sort_in, m, s)) || (rc = grow_dev(&st->sort_out, &st->c_sort_out, m, s))))
        return rc;
    if (m <= kSmallCarry) {
        hipLaunchKernelGGL(small_carry_kernel, dim3(1), dim3(ST), 0, s, st->pairs, (int)m, st->keys[nx], st->grp[nx],
                           st->n_groups + nx);
        HIP_TRY(hipGetLastError());
    } else {
        const int64_t tiles = (m + kSmallCarry - 1) / kSmallCarry;
        hipLaunchKernelGGL(tile_sort_kernel, dim3((unsigned)tiles), dim3(ST), 0, s, st->pairs, m, st->sort_in);
        HIP_TRY(hipGetLastError());
        unsigned long long *src = st->sort_in, *dst = st->sort_out;
        for (int64_t width = kSmallCarry; width < m; width *= 2) {
            const int64_t grid = std::min<int64_t>((m + 255) / 256, 4096);
            hipLaunchKernelGGL(merge_pass_kernel, dim3((unsigned)grid), dim3(256), 0, s, src, dst, m, width);
            HIP_TRY(hipGetLastError());
            std::swap(src, dst);
        }
        hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(ST), 0, s, src, m, st->keys[nx], st->grp[nx],
                           st->n_groups + nx);
        HIP_TRY(hipGetLastError());
    }
    st->cur = nx;
    st->bound = m;
    st->position += n;
    return PFSM_OK;
}

int pfsm_stream_info(pfsm_stream_t *st, int64_t *position, int64_t *n_carried, void *hip_stream) {
    if (!st) return fail(PFSM_EINVAL, "NULL stream");
    if (position) *position = st->position;
    if (n_carried) {
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        int32_t g = 0;
        HIP_TRY(hipMemcpyAsync(&g, st->n_groups + st->cur, sizeof g, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *n_carried = g;
    }
    return PFSM_OK;
}

void pfsm_stream_close(pfsm_stream_t *st) {
    if (!st) return;
    (void)hipDeviceSynchronize();
    delete st;
}

}  // extern "C"
