// Host-side helpers shared by the DFA and NFA halves of libpfsm: error
// reporting, owned device buffers and per-stream scan workspaces.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pfsm.h"
#include "pfsm_dev.h"

namespace pfsmk {

// Thread-local description of the most recent failure (pfsm_last_error).
std::string &last_error();

inline int fail(int code, const char *fmt, ...) {
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error() = buf;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::pfsmk::fail(e_ == hipErrorOutOfMemory ? PFSM_ENOMEM : PFSM_EHIP, "%s: %s (%s:%d)", \
                                 #expr, hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)

// A device buffer owned by a handle.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        HIP_TRY(hipMalloc(&p, n));
        bytes = n;
        return PFSM_OK;
    }
    // Copies `count` elements; the caller synchronises `s` before `src` dies.
    template <typename T>
    int upload(const T *src, size_t count, hipStream_t s) {
        int rc = alloc(count * sizeof(T));
        if (rc) return rc;
        if (count) HIP_TRY(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
        return PFSM_OK;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
    // Copies `count` elements into the buffer as it is (they must fit); the
    // caller synchronises `s` before `src` dies.
    template <typename T>
    int write(const T *src, size_t count, hipStream_t s) {
        if (count * sizeof(T) > bytes) return fail(PFSM_EINVAL, "cache outgrew its buffer");
        if (count) HIP_TRY(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
        return PFSM_OK;
    }
    // Give up ownership of the buffer (the caller frees it later).
    void *detach() {
        void *q = p;
        p = nullptr;
        bytes = 0;
        return q;
    }
};

// Longest stream: positions, shifted by up to 15 bytes for alignment, are
// int32 inside the kernels.
constexpr int64_t kMaxStream = (1ll << 31) - 16;

// Segments a launch may have: inputs are below 2^31 bytes and a segment
// holds at least min(n / grid, 64 KiB) bytes.
constexpr int kMaxSegs = 32768;

// Scan scratch of one handle on one stream: the persistent grid's count
// slots (zeroed once, epoch-tagged afterwards), the segment tickets and
// look-back words, per-workgroup work counters, the device total and pinned
// host mirrors for reading them back.
struct Workspace {
    hipStream_t stream = nullptr;
    int n_blocks = 0;
    int last_grid = 0;                    // workgroups of the last launch
    unsigned long long *slots = nullptr;  // [n_blocks]
    ScanCtl *ctl = nullptr;
    unsigned long long *lb = nullptr;     // [lb_cap]
    int lb_cap = 0;
    void *spill = nullptr;                // DFA: [n_blocks * kDfaSpill] walks
    long long *bstats = nullptr;          // [n_blocks * 4]
    int64_t *h_total = nullptr;           // pinned, mapped
    int64_t *h_total_dev = nullptr;       // h_total's device address
    long long *h_stats = nullptr;         // pinned [n_blocks * 4]
    bool scanned = false;
    uint64_t used = 0;                    // launch sequence number of the last scan
    uint8_t *stage = nullptr;             // aligned copy of a misaligned input
    int64_t stage_cap = 0;
    long long *m_tag = nullptr;           // tag-merged scan: matches per start
    long long *m_seg = nullptr;           //   per segment, then their scan
    int64_t c_m_tag = 0, c_m_seg = 0;
    uint32_t *big_front = nullptr;        // NFA replay frontiers
    uint32_t *big_bits = nullptr;         // NFA replay visited bits (kept clear)
    int64_t big_states = 0;
    MatchOut *defer_rows = nullptr;       // DFA deferred placement: staged rows
    int64_t c_defer_rows = 0;
    long long *defer_seg = nullptr;       //   per segment: first row, count, offset
    int64_t c_defer_seg = 0;
    unsigned long long *defer_cursor = nullptr;
    std::vector<void *> retired;          // replay scratch outgrown by the union

    ~Workspace() {
        for (void *p : retired) (void)hipFree(p);
        if (slots) (void)hipFree(slots);
        if (ctl) (void)hipFree(ctl);
        if (lb) (void)hipFree(lb);
        if (spill) (void)hipFree(spill);
        if (bstats) (void)hipFree(bstats);
        if (h_total) (void)hipHostFree(h_total);
        if (h_stats) (void)hipHostFree(h_stats);
        if (stage) (void)hipFree(stage);
        if (m_tag) (void)hipFree(m_tag);
        if (m_seg) (void)hipFree(m_seg);
        if (big_front) (void)hipFree(big_front);
        if (big_bits) (void)hipFree(big_bits);
        if (defer_rows) (void)hipFree(defer_rows);
        if (defer_seg) (void)hipFree(defer_seg);
        if (defer_cursor) (void)hipFree(defer_cursor);
    }
};

struct WorkspacePool {
    std::mutex mu;
    std::vector<std::unique_ptr<Workspace>> ws;
    uint64_t clock = 0;

    // Record a launch in w (for find()).
    void mark(Workspace *w) {
        std::lock_guard<std::mutex> lk(mu);
        w->scanned = true;
        w->used = ++clock;
    }

    // The workspace of `s`, created on first use for a grid of n_blocks.
    int get(hipStream_t s, int n_blocks, Workspace **out) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &p : ws)
            if (p->stream == s && p->n_blocks == n_blocks) {
                *out = p.get();
                return PFSM_OK;
            }
        auto w = std::make_unique<Workspace>();
        w->stream = s;
        w->n_blocks = n_blocks;
        HIP_TRY(hipMalloc(&w->slots, sizeof(unsigned long long) * n_blocks));
        HIP_TRY(hipMemset(w->slots, 0, sizeof(unsigned long long) * n_blocks));
        HIP_TRY(hipMalloc(&w->ctl, sizeof(ScanCtl)));
        HIP_TRY(hipMemset(w->ctl, 0, sizeof(ScanCtl)));
        w->lb_cap = kMaxSegs + n_blocks;
        HIP_TRY(hipMalloc(&w->lb, sizeof(unsigned long long) * w->lb_cap));
        HIP_TRY(hipMemset(w->lb, 0, sizeof(unsigned long long) * w->lb_cap));
        HIP_TRY(hipMalloc(&w->bstats, sizeof(long long) * 4 * n_blocks));
        HIP_TRY(hipMemset(w->bstats, 0, sizeof(long long) * 4 * n_blocks));
        // The synchronous scan's kernels store the total straight into this
        // mapped, coherent host word: no copy is queued behind the scan.
        HIP_TRY(hipHostMalloc(&w->h_total, sizeof(int64_t), hipHostMallocMapped | hipHostMallocCoherent));
        HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void **>(&w->h_total_dev), w->h_total, 0));
        HIP_TRY(hipHostMalloc(&w->h_stats, sizeof(long long) * 4 * n_blocks, hipHostMallocDefault));
        HIP_TRY(hipDeviceSynchronize());
        *out = w.get();
        ws.push_back(std::move(w));
        return PFSM_OK;
    }

    // The workspace of the most recent scan on `s` (grids of any size).
    Workspace *find(hipStream_t s) {
        std::lock_guard<std::mutex> lk(mu);
        Workspace *r = nullptr;
        for (auto &p : ws)
            if (p->stream == s && p->scanned && (!r || p->used > r->used)) r = p.get();
        return r;
    }
};

// Grow the look-back words of `w` to at least `need` (synchronises the
// stream; the new words are clear, so they carry no epoch in use).
inline int grow_lb(Workspace *w, int need) {
    if (need <= w->lb_cap) return PFSM_OK;
    HIP_TRY(hipStreamSynchronize(w->stream));
    unsigned long long *nb = nullptr;
    HIP_TRY(hipMalloc(&nb, sizeof(unsigned long long) * need));
    HIP_TRY(hipMemset(nb, 0, sizeof(unsigned long long) * need));
    HIP_TRY(hipDeviceSynchronize());
    if (w->lb) HIP_TRY(hipFree(w->lb));
    w->lb = nb;
    w->lb_cap = need;
    return PFSM_OK;
}

// Buffers of the DFA scan's deferred placement: n_segs segments and `rows`
// staged rows at least (grown, never shrunk; the cursor starts at zero).
inline int grow_defer(Workspace *w, int64_t n_segs, int64_t rows) {
    if (n_segs <= w->c_defer_seg && rows <= w->c_defer_rows && w->defer_cursor) return PFSM_OK;
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (!w->defer_cursor) {
        HIP_TRY(hipMalloc(&w->defer_cursor, sizeof(unsigned long long)));
        HIP_TRY(hipMemset(w->defer_cursor, 0, sizeof(unsigned long long)));
    }
    if (n_segs > w->c_defer_seg) {
        const int64_t c = std::max<int64_t>(n_segs, 1024);
        if (w->defer_seg) HIP_TRY(hipFree(w->defer_seg));
        w->defer_seg = nullptr;
        w->c_defer_seg = 0;
        HIP_TRY(hipMalloc(&w->defer_seg, sizeof(long long) * 3 * (size_t)c));
        w->c_defer_seg = c;
    }
    if (rows > w->c_defer_rows) {
        if (w->defer_rows) HIP_TRY(hipFree(w->defer_rows));
        w->defer_rows = nullptr;
        w->c_defer_rows = 0;
        HIP_TRY(hipMalloc(&w->defer_rows, sizeof(MatchOut) * (size_t)rows));
        w->c_defer_rows = rows;
    }
    HIP_TRY(hipDeviceSynchronize());
    return PFSM_OK;
}

// The scan kernels read 16-byte granules and need a 16-byte aligned input:
// a misaligned input is first copied (in stream order) into a buffer of the
// workspace.  *x is replaced by the aligned pointer.
inline int align_input(Workspace *w, const uint8_t **x, int64_t n, hipStream_t s) {
    if ((reinterpret_cast<uintptr_t>(*x) & 15) == 0) return PFSM_OK;
    if (w->stage_cap < n) {
        HIP_TRY(hipStreamSynchronize(s));
        if (w->stage) HIP_TRY(hipFree(w->stage));
        w->stage = nullptr;
        w->stage_cap = 0;
        HIP_TRY(hipMalloc(&w->stage, (size_t)n));
        w->stage_cap = n;
    }
    HIP_TRY(hipMemcpyAsync(w->stage, *x, (size_t)n, hipMemcpyDeviceToDevice, s));
    *x = w->stage;
    return PFSM_OK;
}

// Sum the per-workgroup counters of the last scan in `w` (synchronises).
inline int workspace_stats(Workspace *w, long long v[4]) {
    const int g = w->last_grid;
    for (int k = 0; k < 4; ++k) v[k] = 0;
    if (g <= 0) return PFSM_OK;
    HIP_TRY(hipMemcpyAsync(w->h_stats, w->bstats, sizeof(long long) * 4 * g, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    for (int b = 0; b < g; ++b)
        for (int k = 0; k < 4; ++k) v[k] += w->h_stats[4 * b + k];
    return PFSM_OK;
}

// Compute units of the current device.
int device_cus(int *out);

// Tuning knobs of a handle (pfsm_set_option); 0 / -1 select the defaults.
struct Knobs {
    int64_t segment = 0;       // bytes per segment cap
    int32_t wpc = 0;           // workgroups per compute unit
    int64_t table_budget = -1; // DFA: largest LDS-resident table
    int32_t pair_cache = 1;    // NFA: two-symbol cache allowed
    int32_t merged = 0;        // DFA: tag-merged stepping
    int32_t merged_lim = 0;    // DFA, tag-merged: 32-bit count limit (0 = 2^31 - 1)
};

// Resident workgroups of a launch: `wpc` per compute unit (at most the
// occupancy limit `occ`; 0 = occ).
inline int grid_blocks(int occ, int cus, int wpc) {
    const int k = wpc > 0 && wpc < occ ? wpc : occ;
    return k * cus;
}

// Split n bytes over a persistent grid of n_blocks workgroups: bytes per
// workgroup and round (a multiple of 16) and the number of rounds.
// Segments are n / n_blocks bytes, at least seg_floor and at most
// seg_target (a multiple of 16).  Small DFA inputs use a 4 KiB floor (four
// slices): below it a segment's fixed work (start-up, ticket, look-back)
// outweighs its walks, which run one start per lane.  NFA inputs keep
// 16-byte segments, because a start whose state set outgrows a lane is
// replayed by its whole workgroup, one start at a time, so starts spread
// over more workgroups replay in parallel.
constexpr int64_t kDfaSegFloor = 4096;
// Inputs of at most 16 KiB scanned with an LDS image of at most 16 KiB (a
// small table) take 256-byte segments instead: the image loads quickly, so
// more workgroups shorten the scan (4 KiB against a 16-state DFA: 23 to
// 18.5 us of kernel time).  With a large image the extra start-ups cost as
// much as they save.
constexpr int64_t kDfaSegFloorSmall = 256;
constexpr int64_t kDfaSmallInput = 16384;
constexpr int32_t kDfaSmallImage = 16384;
inline int64_t dfa_seg_floor(int64_t n, int32_t image_bytes) {
    return n <= kDfaSmallInput && image_bytes <= kDfaSmallImage ? kDfaSegFloorSmall : kDfaSegFloor;
}
constexpr int64_t kNfaSegFloor = 16;

inline void plan_segments(int64_t n, int n_blocks, int64_t seg_target, int64_t seg_floor, int64_t *seg, int *rounds) {
    int64_t per = (n + n_blocks - 1) / n_blocks;
    per = (per + 15) / 16 * 16;
    if (per < seg_floor) per = seg_floor;
    if (per > seg_target) per = seg_target;
    *seg = per;
    *rounds = (int)((n + per * n_blocks - 1) / (per * n_blocks));
    if (*rounds < 1) *rounds = 1;
}

}  // namespace pfsmk
