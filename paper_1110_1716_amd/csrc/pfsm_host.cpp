// Host side of libpfsm: descriptor validation, the read-only caches derived
// from an automaton, device upload, per-stream scan workspaces and the C ABI
// declared in include/pfsm.h.
#include "pfsm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pfsm_dev.h"
#include "pfsm_nfa.h"

using namespace pfsmk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(PFSM_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                        __FILE__, __LINE__);                                            \
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
        if (n == 0) n = 1;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(e == hipErrorOutOfMemory ? PFSM_ENOMEM : PFSM_EHIP, "hipMalloc(%zu): %s", n,
                        hipGetErrorString(e));
        }
        bytes = n;
        return PFSM_OK;
    }
    template <typename T>
    int upload(const T *src, size_t count, hipStream_t s) {
        int rc = alloc(count * sizeof(T));
        if (rc) return rc;
        if (count) HIP_TRY(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
        return PFSM_OK;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Scan scratch for one stream: look-back status words, the control block,
// the device total and a pinned host slot for reading it back.
struct Workspace {
    hipStream_t stream = nullptr;
    ScanCtl *ctl = nullptr;
    unsigned long long *status = nullptr;
    int64_t status_cap = 0;
    int64_t *d_total = nullptr;
    int64_t *h_total = nullptr;
    long long *h_last = nullptr;
    bool scanned = false;
    std::vector<void *> extra;  // kernel-specific scratch, freed with the workspace

    ~Workspace() {
        if (ctl) (void)hipFree(ctl);
        if (status) (void)hipFree(status);
        if (d_total) (void)hipFree(d_total);
        if (h_total) (void)hipHostFree(h_total);
        if (h_last) (void)hipHostFree(h_last);
        for (void *p : extra) (void)hipFree(p);
    }
};

}  // namespace

struct pfsm {
    int kind = 0;  // 0 = DFA, 1 = NFA
    // ---- DFA: host copy (used to rebuild caches when a label is removed)
    int32_t n_states = 0, n_symbols = 0, q0 = 0;
    bool identity = true;
    std::vector<int16_t> b2s;       // [256]
    std::vector<int32_t> delta;     // [n_states * n_symbols]
    std::vector<std::vector<int32_t>> labels;  // per state: sorted unique labels
    std::vector<int32_t> disabled;  // removed labels (sorted)
    // ---- DFA: device
    DevBuf d_tbl, d_b2s, d_first, d_flags, d_lab_off, d_lab;
    bool tbl16 = true;
    // ---- NFA
    NfaPtr nfa;
    // ---- workspaces
    std::mutex ws_mu;
    std::vector<std::unique_ptr<Workspace>> ws;
};

namespace {

// ------------------------------------------------------------------ workspaces

int get_workspace(pfsm_t *h, hipStream_t s, int64_t n_windows, Workspace **out) {
    std::lock_guard<std::mutex> lk(h->ws_mu);
    Workspace *w = nullptr;
    for (auto &p : h->ws)
        if (p->stream == s) w = p.get();
    if (!w) {
        auto nw = std::make_unique<Workspace>();
        nw->stream = s;
        HIP_TRY(hipMalloc(&nw->ctl, sizeof(ScanCtl)));
        HIP_TRY(hipMemset(nw->ctl, 0, sizeof(ScanCtl)));
        HIP_TRY(hipMalloc(&nw->d_total, sizeof(int64_t)));
        HIP_TRY(hipHostMalloc(&nw->h_total, sizeof(int64_t), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc(&nw->h_last, 4 * sizeof(long long), hipHostMallocDefault));
        HIP_TRY(hipDeviceSynchronize());
        w = nw.get();
        h->ws.push_back(std::move(nw));
    }
    if (n_windows > w->status_cap) {
        // Earlier launches on this stream may still read the old array.
        HIP_TRY(hipStreamSynchronize(s));
        if (w->status) HIP_TRY(hipFree(w->status));
        w->status = nullptr;
        int64_t cap = std::max<int64_t>(n_windows, 1024);
        hipError_t e = hipMalloc(&w->status, cap * sizeof(unsigned long long));
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? PFSM_ENOMEM : PFSM_EHIP, "status alloc: %s",
                        hipGetErrorString(e));
        HIP_TRY(hipMemset(w->status, 0, cap * sizeof(unsigned long long)));
        HIP_TRY(hipDeviceSynchronize());
        w->status_cap = cap;
    }
    *out = w;
    return PFSM_OK;
}

// ------------------------------------------------------------------ validation helpers

int check_labels(int32_t n_states, const int32_t *off, const int32_t *lab) {
    if (!off) return fail(PFSM_EINVAL, "final_off is NULL");
    if (off[0] != 0) return fail(PFSM_EINVAL, "final_off[0] must be 0");
    for (int32_t q = 0; q < n_states; ++q)
        if (off[q + 1] < off[q]) return fail(PFSM_EINVAL, "final_off decreases at state %d", q);
    const int32_t nnz = off[n_states];
    if (nnz > 0 && !lab) return fail(PFSM_EINVAL, "final_labels is NULL");
    for (int32_t i = 0; i < nnz; ++i)
        if (lab[i] < 0) return fail(PFSM_EINVAL, "label %d is negative", lab[i]);
    return PFSM_OK;
}

std::vector<std::vector<int32_t>> label_sets(int32_t n_states, const int32_t *off, const int32_t *lab) {
    std::vector<std::vector<int32_t>> out(n_states);
    for (int32_t q = 0; q < n_states; ++q) {
        auto &v = out[q];
        v.assign(lab + off[q], lab + off[q + 1]);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    return out;
}

bool has_label(const std::vector<int32_t> &sorted, int32_t l) {
    return std::binary_search(sorted.begin(), sorted.end(), l);
}

// ------------------------------------------------------------------ DFA caches

// Rebuild and upload the caches that depend on the enabled label sets:
// live flags (reverse search from states with an enabled label over
// transitions that some byte can take), the q0 row per byte, label CSR.
int dfa_upload_caches(pfsm_t *h, hipStream_t s) {
    const int32_t N = h->n_states, S = h->n_symbols;
    std::vector<std::vector<int32_t>> en(N);
    for (int32_t q = 0; q < N; ++q)
        for (int32_t l : h->labels[q])
            if (!has_label(h->disabled, l)) en[q].push_back(l);

    std::vector<uint8_t> sym_used(S, 0);
    for (int b = 0; b < 256; ++b)
        if (h->b2s[b] >= 0) sym_used[h->b2s[b]] = 1;
    // reverse adjacency
    std::vector<int32_t> roff(N + 1, 0);
    for (int64_t i = 0; i < (int64_t)N * S; ++i)
        if (h->delta[i] >= 0 && sym_used[i % S]) roff[h->delta[i] + 1]++;
    for (int32_t q = 0; q < N; ++q) roff[q + 1] += roff[q];
    std::vector<int32_t> radj(roff[N]), fillp(roff.begin(), roff.end() - 1);
    for (int64_t i = 0; i < (int64_t)N * S; ++i)
        if (h->delta[i] >= 0 && sym_used[i % S]) radj[fillp[h->delta[i]]++] = (int32_t)(i / S);
    std::vector<uint8_t> flags(N, 0);
    std::vector<int32_t> queue;
    queue.reserve(N);
    for (int32_t q = 0; q < N; ++q)
        if (!en[q].empty()) {
            flags[q] = kLive | kFinal;
            queue.push_back(q);
        }
    for (size_t i = 0; i < queue.size(); ++i)
        for (int32_t k = roff[queue[i]]; k < roff[queue[i] + 1]; ++k)
            if (!(flags[radj[k]] & kLive)) {
                flags[radj[k]] |= kLive;
                queue.push_back(radj[k]);
            }
    std::vector<int32_t> first(256, -1);
    for (int b = 0; b < 256; ++b) {
        int sym = h->b2s[b];
        if (sym < 0) continue;
        int32_t t = h->delta[(int64_t)h->q0 * S + sym];
        if (t >= 0 && (flags[t] & kLive)) first[b] = t;
    }
    std::vector<int32_t> off(N + 1, 0), lab;
    for (int32_t q = 0; q < N; ++q) {
        lab.insert(lab.end(), en[q].begin(), en[q].end());
        off[q + 1] = (int32_t)lab.size();
    }
    int rc;
    if ((rc = h->d_first.upload(first.data(), 256, s))) return rc;
    if ((rc = h->d_flags.upload(flags.data(), N, s))) return rc;
    if ((rc = h->d_lab_off.upload(off.data(), N + 1, s))) return rc;
    if ((rc = h->d_lab.upload(lab.data(), lab.size(), s))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return PFSM_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char *pfsm_strerror(int code) {
    switch (code) {
    case PFSM_OK: return "success";
    case PFSM_EINVAL: return "invalid argument or descriptor";
    case PFSM_ENOMEM: return "out of memory";
    case PFSM_EOVERFLOW: return "more matches than the output capacity";
    case PFSM_EHIP: return "HIP runtime error";
    case PFSM_ENOENT: return "no pattern carries the label";
    case PFSM_EEXIST: return "label already present";
    case PFSM_ENOSYS: return "operation not supported for this handle";
    default: return "unknown error";
    }
}

const char *pfsm_last_error(void) { return g_err.c_str(); }

int pfsm_load_dfa(pfsm_t **out, const pfsm_dfa_desc *d, void *hip_stream) {
    if (!out || !d) return fail(PFSM_EINVAL, "NULL argument");
    *out = nullptr;
    const int32_t N = d->n_states, S = d->n_symbols;
    if (N < 1 || S < 1) return fail(PFSM_EINVAL, "n_states and n_symbols must be >= 1");
    if ((int64_t)N * S >= (1ll << 31)) return fail(PFSM_EINVAL, "n_states * n_symbols must be < 2^31");
    if (d->q0 < 0 || d->q0 >= N) return fail(PFSM_EINVAL, "q0 out of range");
    if (!d->byte_to_symbol && S != 256)
        return fail(PFSM_EINVAL, "byte_to_symbol may be NULL only when n_symbols == 256");
    if (!d->delta) return fail(PFSM_EINVAL, "delta is NULL");
    for (int64_t i = 0; i < (int64_t)N * S; ++i)
        if (d->delta[i] < -1 || d->delta[i] >= N)
            return fail(PFSM_EINVAL, "delta[%lld] = %d out of range", (long long)i, d->delta[i]);
    if (d->byte_to_symbol)
        for (int b = 0; b < 256; ++b)
            if (d->byte_to_symbol[b] < -1 || d->byte_to_symbol[b] >= S)
                return fail(PFSM_EINVAL, "byte_to_symbol[%d] out of range", b);
    int rc = check_labels(N, d->final_off, d->final_labels);
    if (rc) return rc;

    std::unique_ptr<pfsm_t> h(new (std::nothrow) pfsm_t);
    if (!h) return fail(PFSM_ENOMEM, "handle");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    h->kind = 0;
    h->n_states = N;
    h->n_symbols = S;
    h->q0 = d->q0;
    h->identity = d->byte_to_symbol == nullptr;
    h->b2s.resize(256);
    for (int b = 0; b < 256; ++b) h->b2s[b] = d->byte_to_symbol ? d->byte_to_symbol[b] : (int16_t)b;
    h->delta.assign(d->delta, d->delta + (int64_t)N * S);
    h->labels = label_sets(N, d->final_off, d->final_labels);
    h->tbl16 = N <= 32767;
    if (h->tbl16) {
        std::vector<int16_t> t16(h->delta.begin(), h->delta.end());
        if ((rc = h->d_tbl.upload(t16.data(), t16.size(), s))) return rc;
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        if ((rc = h->d_tbl.upload(h->delta.data(), h->delta.size(), s))) return rc;
    }
    if ((rc = h->d_b2s.upload(h->b2s.data(), 256, s))) return rc;
    if ((rc = dfa_upload_caches(h.get(), s))) return rc;
    *out = h.release();
    return PFSM_OK;
}

int pfsm_load_nfa(pfsm_t **out, const pfsm_nfa_desc *d, void *hip_stream) {
    if (!out || !d) return fail(PFSM_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_ptr<pfsm_t> h(new (std::nothrow) pfsm_t);
    if (!h) return fail(PFSM_ENOMEM, "handle");
    h->kind = 1;
    std::string err;
    int rc = nfa_load(d, static_cast<hipStream_t>(hip_stream), &h->nfa, &err);
    if (rc) return fail(rc, "%s", err.c_str());
    *out = h.release();
    return PFSM_OK;
}

int pfsm_add_pattern(pfsm_t *h, const pfsm_nfa_desc *pattern, void *hip_stream) {
    if (!h || !pattern) return fail(PFSM_EINVAL, "NULL argument");
    if (h->kind == 0)
        return fail(PFSM_ENOSYS, "a DFA handle is one monolithic table; load the union as an NFA");
    std::string err;
    int rc = nfa_add_pattern(h->nfa.get(), pattern, static_cast<hipStream_t>(hip_stream), &err);
    if (rc) return fail(rc, "%s", err.c_str());
    return PFSM_OK;
}

int pfsm_remove_pattern(pfsm_t *h, int32_t label, void *hip_stream) {
    if (!h) return fail(PFSM_EINVAL, "NULL handle");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (h->kind == 1) {
        std::string err;
        int rc = nfa_remove_pattern(h->nfa.get(), label, s, &err);
        if (rc) return fail(rc, "%s", err.c_str());
        return PFSM_OK;
    }
    if (has_label(h->disabled, label)) return fail(PFSM_ENOENT, "label %d already removed", label);
    bool found = false;
    for (auto &v : h->labels)
        if (has_label(v, label)) { found = true; break; }
    if (!found) return fail(PFSM_ENOENT, "no final state carries label %d", label);
    h->disabled.insert(std::upper_bound(h->disabled.begin(), h->disabled.end(), label), label);
    // Scans already on the stream read the current caches; wait for them,
    // then replace the caches in place.
    HIP_TRY(hipStreamSynchronize(s));
    return dfa_upload_caches(h, s);
}

static int choose_per_thread(int64_t n) {
    // Windows of 256 * B bytes; keep enough windows to fill 256 CUs.
    if (n >= (int64_t)4096 * 256 * 4) return 16;
    if (n >= (int64_t)1024 * 256 * 4) return 4;
    return 1;
}

int pfsm_scan_async(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
                    int64_t *d_n_matches, void *hip_stream) {
    if (!h) return fail(PFSM_EINVAL, "NULL handle");
    if (n < 0 || n >= (1ll << 31)) return fail(PFSM_EINVAL, "n must be in [0, 2^31)");
    if (cap < 0) return fail(PFSM_EINVAL, "cap must be >= 0");
    if (!d_n_matches) return fail(PFSM_EINVAL, "d_n_matches is NULL");
    if (n > 0 && !d_input) return fail(PFSM_EINVAL, "d_input is NULL");
    if (cap > 0 && !d_out) return fail(PFSM_EINVAL, "d_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (n == 0) {
        HIP_TRY(launch_write_zero(d_n_matches, s));
        return PFSM_OK;
    }
    if (h->kind == 1) {
        std::string err;
        int rc = nfa_scan_async(h->nfa.get(), d_input, n, reinterpret_cast<MatchOut *>(d_out), cap,
                                d_n_matches, s, &err);
        if (rc) return fail(rc, "%s", err.c_str());
        return PFSM_OK;
    }
    const int B = choose_per_thread(n);
    const int64_t W = (int64_t)kBlock * B;
    const int64_t G = (n + W - 1) / W;
    Workspace *w;
    int rc = get_workspace(h, s, G, &w);
    if (rc) return rc;
    DfaArgs a;
    a.x = d_input;
    a.n = n;
    a.tbl = h->d_tbl.p;
    a.n_states = h->n_states;
    a.n_symbols = h->n_symbols;
    a.b2s = h->d_b2s.as<int16_t>();
    a.first = h->d_first.as<int32_t>();
    a.flags = h->d_flags.as<uint8_t>();
    a.lab_off = h->d_lab_off.as<int32_t>();
    a.lab = h->d_lab.as<int32_t>();
    a.out = reinterpret_cast<MatchOut *>(d_out);
    a.cap = cap;
    a.total = d_n_matches;
    a.ctl = w->ctl;
    a.status = w->status;
    a.n_windows = (int32_t)G;
    HIP_TRY(launch_dfa_scan(a, B, h->identity, h->tbl16, s));
    w->scanned = true;
    return PFSM_OK;
}

int pfsm_scan(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
              int64_t *n_matches, void *hip_stream) {
    if (!h || !n_matches) return fail(PFSM_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Workspace *w;
    int rc = get_workspace(h, s, 0, &w);
    if (rc) return rc;
    rc = pfsm_scan_async(h, d_input, n, d_out, cap, w->d_total, hip_stream);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(w->h_total, w->d_total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_matches = *w->h_total;
    if (*n_matches > cap)
        return fail(PFSM_EOVERFLOW, "%lld matches, capacity %lld", (long long)*n_matches, (long long)cap);
    return PFSM_OK;
}

int pfsm_scan_batch(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data,
                    const int64_t *d_stream_off, const int32_t *d_stream_automaton, int32_t n_streams,
                    pfsm_match_t *d_out, int64_t cap, int64_t *d_match_off, int64_t *n_matches,
                    void *hip_stream) {
    (void)hs; (void)n_automata; (void)d_data; (void)d_stream_off; (void)d_stream_automaton;
    (void)n_streams; (void)d_out; (void)cap; (void)d_match_off; (void)n_matches; (void)hip_stream;
    return fail(PFSM_ENOSYS, "pfsm_scan_batch is not available yet");
}

int pfsm_last_stats(pfsm_t *h, pfsm_stats *out, void *hip_stream) {
    if (!h || !out) return fail(PFSM_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(h->ws_mu);
        for (auto &p : h->ws)
            if (p->stream == s) w = p.get();
    }
    if (h->kind == 1) {
        std::string err;
        long long v[4];
        int rc = nfa_last_stats(h->nfa.get(), s, v, &err);
        if (rc) return fail(rc, "%s", err.c_str());
        out->transitions = v[0]; out->activations = v[1]; out->long_walks = v[2]; out->matches = v[3];
        return PFSM_OK;
    }
    if (!w || !w->scanned) return fail(PFSM_ENOENT, "no scan on this stream yet");
    HIP_TRY(hipMemcpyAsync(w->h_last, w->ctl->last, 4 * sizeof(long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->transitions = w->h_last[0];
    out->activations = w->h_last[1];
    out->long_walks = w->h_last[2];
    out->matches = w->h_last[3];
    return PFSM_OK;
}

void pfsm_free(pfsm_t *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

}  // extern "C"
