// Serving loop: continuous batching of scan requests against resident
// automata (the online use of Section I: matches are reported for streams as
// they come in).
//
// One worker thread owns the device side.  Requests wait in a FIFO; the
// worker packs as many as fit the memory budget (their bytes plus an output
// estimate) into a free slot and enqueues the whole batch on that slot's
// stream (planning, one scan launch per automaton, offsets, gather; see
// batch.hip), then goes on admitting into the other slot while the first
// batch runs.  The slots' kernels run in launch order, so batches finish in
// turn and each slot is refilled while the other computes.  When a slot's
// batch is done its matches are copied back, the
// slot takes its next batch, and only then are the matches handed to the
// waiting callers.  A batch whose output outgrows the
// estimate is run again at the exact size (the total is known by then).
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "host_common.h"
#include "pfsm.h"

using namespace pfsmk;

namespace {

constexpr int kSlots = 2;
constexpr int64_t kBatchBytes = 32ll << 20;  // input bytes per batch (two batches pipeline)

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

struct Req {
    int64_t id = 0;
    int64_t t_submit = 0, t_done = 0;  // CLOCK_MONOTONIC ns
    int32_t aut = 0;
    std::vector<uint8_t> bytes;  // a copy, or empty when borrowed
    const uint8_t *src = nullptr;  // the request's bytes (bytes.data() or the caller's)
    int64_t n = 0;
    int64_t exact = -1;  // its match count, once a batch has counted it
    // its matches: rows of its batch's pinned output buffer, which it keeps
    // alive (shared with the batch's other requests) until it is released
    const pfsm_match_t *result = nullptr;
    std::shared_ptr<struct OutBuf> hold;
    int64_t n_result = 0;
    int status = PFSM_OK;
    bool done = false;
};

// Threads that share the host copies of a batch (packing inputs, handing
// out results): run(n, f) calls f(0..n-1) on the pool and the caller.
class CopyPool {
  public:
    explicit CopyPool(int n_threads) {
        for (int t = 0; t < n_threads; ++t) th_.emplace_back([this] { loop(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    void run(int n, const std::function<void(int)> &f) {
        if (n <= 0) return;
        {
            std::lock_guard<std::mutex> lk(m_);
            f_ = &f;
            n_ = n;
            next_ = 0;
            done_ = 0;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(m_);
        cv_done_.wait(lk, [&] { return done_ == n_; });
        f_ = nullptr;
    }

  private:
    void work() {
        for (;;) {
            int i;
            const std::function<void(int)> *f;
            {
                std::lock_guard<std::mutex> lk(m_);
                if (!f_ || next_ >= n_) return;
                i = next_++;
                f = f_;
            }
            (*f)(i);
            std::lock_guard<std::mutex> lk(m_);
            if (++done_ == n_) cv_done_.notify_all();
        }
    }
    void loop() {
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || (f_ && next_ < n_); });
                if (stop_) return;
            }
            work();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, cv_done_;
    const std::function<void(int)> *f_ = nullptr;
    int n_ = 0, next_ = 0, done_ = 0;
    bool stop_ = false;
};

constexpr int kCopyThreads = 7;         // helpers besides the worker
constexpr int64_t kCopyChunk = 1 << 20;  // bytes per copy task

// A buffer that only grows (contents are not kept).
struct Buf {
    void *p = nullptr;
    int64_t cap = 0;
    bool pinned = false;
    int reserve(int64_t need) {
        if (need <= cap) return PFSM_OK;
        release();
        const int64_t n = std::max<int64_t>(need, 256);
        if (pinned) HIP_TRY(hipHostMalloc(&p, (size_t)n, hipHostMallocDefault));
        else HIP_TRY(hipMalloc(&p, (size_t)n));
        cap = n;
        return PFSM_OK;
    }
    void release() {
        if (p) (void)(pinned ? hipHostFree(p) : hipFree(p));
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

// A pinned buffer that receives one batch's output.  The batch's requests
// point into it and share it; when the last of them is released it goes
// back to the pool for a later batch.
struct OutBuf {
    void *p = nullptr;
    int64_t cap = 0;  // bytes
};

constexpr int64_t kOutMin = 32ll << 20;  // smallest output buffer allocated, bytes

class OutPool {
  public:
    ~OutPool() {
        for (OutBuf *b : all_) {
            if (b->p) (void)hipHostFree(b->p);
            delete b;
        }
    }
    // An idle buffer of at least `bytes`, else a new one.
    int get(int64_t bytes, std::shared_ptr<OutBuf> *out) {
        OutBuf *b = nullptr;
        {
            std::lock_guard<std::mutex> lk(m_);
            for (size_t i = 0; i < free_.size(); ++i)
                if (free_[i]->cap >= bytes) {
                    b = free_[i];
                    free_[i] = free_.back();
                    free_.pop_back();
                    break;
                }
        }
        if (!b) {
            std::unique_ptr<OutBuf> nb(new (std::nothrow) OutBuf);
            if (!nb) return fail(PFSM_ENOMEM, "out of host memory");
            const int64_t n = std::max<int64_t>(bytes, kOutMin);
            HIP_TRY(hipHostMalloc(&nb->p, (size_t)n, hipHostMallocDefault));
            nb->cap = n;
            b = nb.release();
            std::lock_guard<std::mutex> lk(m_);
            all_.push_back(b);
        }
        *out = std::shared_ptr<OutBuf>(b, [this](OutBuf *x) {
            std::lock_guard<std::mutex> lk(m_);
            free_.push_back(x);
        });
        return PFSM_OK;
    }

  private:
    std::mutex m_;
    std::vector<OutBuf *> free_, all_;
};

// Host and device buffers of one batch in flight.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipEvent_t kdone = nullptr;  // the batch's kernels have ended
    bool busy = false;
    std::vector<Req *> reqs;
    int64_t bytes = 0;    // input bytes of this batch
    int64_t out_cap = 0;  // output rows reserved for it
    Buf h_data{nullptr, 0, true}, h_off{nullptr, 0, true}, h_aut{nullptr, 0, true}, h_moff{nullptr, 0, true},
        h_info{nullptr, 0, true}, h_lohi{nullptr, 0, true};
    // The batch copies its whole output reservation to the host in stream
    // order, into a pinned buffer from the pool that its requests keep.
    std::shared_ptr<OutBuf> h_out;
    Buf d_data, d_off, d_aut, d_moff, d_out;
    BatchRun run;

    void release() {
        for (Buf *b : {&h_data, &h_off, &h_aut, &h_moff, &h_info, &h_lohi, &d_data, &d_off, &d_aut, &d_moff, &d_out})
            b->release();
        h_out.reset();
        if (ev) (void)hipEventDestroy(ev);
        if (kdone) (void)hipEventDestroy(kdone);
        if (stream) (void)hipStreamDestroy(stream);
        ev = nullptr;
        kdone = nullptr;
        stream = nullptr;
    }
};

}  // namespace

struct pfsm_server {
    OutPool out_pool;  // first: outlives the requests and slots that share its buffers
    std::vector<pfsm_t *> hs;
    int device = 0;
    int64_t budget = 0;
    int32_t max_batch = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> queue;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    int64_t next_id = 1;
    bool stop = false;
    Slot slots[kSlots];
    hipEvent_t last_kdone = nullptr;  // kernels of the batch launched last (worker thread only)
    std::thread worker;
    int64_t inflight = 0;  // bytes charged to busy slots (worker thread only)
    pfsm_server_stats st{};
    std::vector<double> density;  // matches per byte seen so far, per automaton (worker only)
    std::unique_ptr<CopyPool> pool;

    // Copy many (dst, src, bytes) pieces, split in chunks over the pool.
    void copy_all(const std::vector<std::tuple<void *, const void *, int64_t>> &parts) {
        std::vector<std::tuple<char *, const char *, int64_t>> chunks;
        int64_t total = 0;
        for (auto &p : parts) {
            char *d = static_cast<char *>(std::get<0>(p));
            const char *s = static_cast<const char *>(std::get<1>(p));
            for (int64_t o = 0; o < std::get<2>(p); o += kCopyChunk)
                chunks.emplace_back(d + o, s + o, std::min(kCopyChunk, std::get<2>(p) - o));
            total += std::get<2>(p);
        }
        if (total < (4 << 20)) {
            for (auto &c : chunks) std::memcpy(std::get<0>(c), std::get<1>(c), (size_t)std::get<2>(c));
            return;
        }
        pool->run((int)chunks.size(), [&](int i) {
            std::memcpy(std::get<0>(chunks[i]), std::get<1>(chunks[i]), (size_t)std::get<2>(chunks[i]));
        });
    }

    // Output rows to reserve for a request: its count when a batch has
    // counted it, else its automaton's density so far with a margin.
    int64_t out_estimate(const Req *r) const {
        if (r->exact >= 0) return r->exact;
        return (int64_t)((double)r->n * density[r->aut] * 1.5) + 256;
    }
    static int64_t charge(int64_t bytes, int64_t out_rows) {
        return bytes + out_rows * (int64_t)(sizeof(pfsm_match_t) * 2);
    }

    void finish(Slot &sl, int status) {
        {
            std::lock_guard<std::mutex> lk(mu);
            const int64_t t = now_ns();
            for (Req *r : sl.reqs) {
                if (status != PFSM_OK) r->status = status;
                r->t_done = t;
                r->done = true;
            }
            st.requests += (int64_t)sl.reqs.size();
            st.bytes += sl.bytes;
        }
        cv_done.notify_all();
        inflight -= charge(sl.bytes, sl.out_cap);
        sl.reqs.clear();
        sl.busy = false;
    }

    // Copy the slot's requests into its buffers and enqueue the batch.
    int launch(Slot &sl) {
        const int64_t nr = (int64_t)sl.reqs.size();
        int rc;
        if ((rc = sl.h_data.reserve(sl.bytes))) return rc;
        if ((rc = sl.d_data.reserve(sl.bytes + 16))) return rc;
        if ((rc = sl.h_off.reserve(8 * (nr + 1)))) return rc;
        if ((rc = sl.d_off.reserve(8 * (nr + 1)))) return rc;
        if ((rc = sl.h_moff.reserve(8 * (nr + 1)))) return rc;
        if ((rc = sl.d_moff.reserve(8 * (nr + 1)))) return rc;
        if ((rc = sl.h_aut.reserve(4 * nr))) return rc;
        if ((rc = sl.d_aut.reserve(4 * nr))) return rc;
        if ((rc = sl.d_out.reserve(sl.out_cap * (int64_t)sizeof(MatchOut)))) return rc;
        if ((rc = out_pool.get(std::max<int64_t>(sl.out_cap, 1) * (int64_t)sizeof(MatchOut), &sl.h_out))) return rc;
        if ((rc = sl.h_info.reserve(sizeof(BatchInfo)))) return rc;
        const int64_t t0 = now_ns();
        int64_t pos = 0;
        std::vector<std::tuple<void *, const void *, int64_t>> parts;
        parts.reserve(nr);
        for (int64_t j = 0; j < nr; ++j) {
            Req *r = sl.reqs[j];
            sl.h_off.as<int64_t>()[j] = pos;
            sl.h_aut.as<int32_t>()[j] = r->aut;
            if (r->n) parts.emplace_back(sl.h_data.as<uint8_t>() + pos, r->src, r->n);
            pos += r->n;
        }
        copy_all(parts);
        sl.h_off.as<int64_t>()[nr] = pos;
        const int64_t t1 = now_ns();
        if (pos) HIP_TRY(hipMemcpyAsync(sl.d_data.p, sl.h_data.p, pos, hipMemcpyHostToDevice, sl.stream));
        HIP_TRY(hipMemcpyAsync(sl.d_off.p, sl.h_off.p, 8 * (nr + 1), hipMemcpyHostToDevice, sl.stream));
        HIP_TRY(hipMemcpyAsync(sl.d_aut.p, sl.h_aut.p, 4 * nr, hipMemcpyHostToDevice, sl.stream));
        // Batches compute in launch order: this batch's kernels start when
        // those of the batch launched before it have ended (its input copy
        // still overlaps them).  Batches then finish one after another, and
        // the worker refills each slot while the next batch computes.
        if (last_kdone && last_kdone != sl.kdone) HIP_TRY(hipStreamWaitEvent(sl.stream, last_kdone, 0));
        if ((rc = batch_run(hs.data(), (int32_t)hs.size(), sl.d_data.as<uint8_t>(), sl.d_off.as<int64_t>(),
                            sl.d_aut.as<int32_t>(), (int32_t)nr, sl.d_out.as<MatchOut>(), sl.out_cap,
                            sl.d_moff.as<int64_t>(), sl.stream, &sl.run)))
            return rc;
        HIP_TRY(hipEventRecord(sl.kdone, sl.stream));
        last_kdone = sl.kdone;
        HIP_TRY(hipMemcpyAsync(sl.h_moff.p, sl.d_moff.p, 8 * (nr + 1), hipMemcpyDeviceToHost, sl.stream));
        HIP_TRY(hipMemcpyAsync(sl.h_info.p, sl.run.info, sizeof(BatchInfo), hipMemcpyDeviceToHost, sl.stream));
        if (sl.out_cap > 0)
            HIP_TRY(hipMemcpyAsync(sl.h_out->p, sl.d_out.p, sl.out_cap * (int64_t)sizeof(MatchOut),
                                   hipMemcpyDeviceToHost, sl.stream));
        HIP_TRY(hipEventRecord(sl.ev, sl.stream));
        std::lock_guard<std::mutex> lk(mu);
        ++st.batches;
        st.pack_ns += t1 - t0;
        st.launch_ns += now_ns() - t1;
        return PFSM_OK;
    }

    // The slot's batch has finished: deliver the results of every request
    // whose matches are all in the output; the others (the output estimate
    // was short) go back to the front of the queue with their exact count.
    int complete(Slot &sl) {
        const int64_t nr = (int64_t)sl.reqs.size();
        const BatchInfo info = *sl.h_info.as<BatchInfo>();
        bool again = false;
        int rc = batch_fit(&sl.run, info, sl.stream, &again);
        if (rc) return rc;
        if (again) {
            {
                std::lock_guard<std::mutex> lk(mu);
                ++st.reruns;
            }
            return launch(sl);
        }
        const int64_t *mo = sl.h_moff.as<int64_t>();
        const int64_t total = mo[nr];
        std::vector<char> whole(nr, 1);
        if (total > sl.out_cap) {
            // a request is whole when its output rows and its stage rows fit
            if ((rc = sl.h_lohi.reserve(16 * nr))) return rc;
            int64_t *hi = sl.h_lohi.as<int64_t>();
            HIP_TRY(hipMemcpyAsync(hi, sl.run.stream_hi, 8 * nr, hipMemcpyDeviceToHost, sl.stream));
            HIP_TRY(hipStreamSynchronize(sl.stream));
            for (int64_t j = 0; j < nr; ++j) whole[j] = mo[j + 1] <= sl.out_cap && hi[j] <= sl.run.stage_cap;
        }
        const int64_t t0 = now_ns();
        // the batch's output rows, min(total, out_cap), are in h_out: each
        // whole request's results are its rows there
        const pfsm_match_t *m = static_cast<const pfsm_match_t *>(sl.h_out->p);
        std::vector<Req *> redo;
        std::vector<Req *> done;
        for (int64_t j = 0; j < nr; ++j) {
            Req *r = sl.reqs[j];
            const int64_t k = mo[j + 1] - mo[j];
            if (r->n > 0) {
                const double d = (double)k / (double)r->n;
                density[r->aut] = std::max(d, 0.8 * density[r->aut] + 0.2 * d);
            }
            if (whole[j]) {
                r->result = k ? m + mo[j] : nullptr;
                if (k) r->hold = sl.h_out;
                r->n_result = k;
                done.push_back(r);
            } else {
                r->exact = k;
                redo.push_back(r);
            }
        }
        if (!redo.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            for (auto it = redo.rbegin(); it != redo.rend(); ++it) queue.push_front(*it);
            ++st.reruns;
        }
        // Hand the slot to the next batch: its inputs and device buffers are
        // free now, and the matches stay in the output buffer the requests
        // hold.
        const int64_t t1 = now_ns();
        const int64_t bytes = sl.bytes;
        inflight -= charge(bytes, sl.out_cap);
        sl.reqs.clear();
        sl.busy = false;
        sl.h_out.reset();
        if (admit(sl)) {
            sl.busy = true;
            const int lrc = launch(sl);
            if (lrc) finish(sl, lrc);
        }
        const int64_t t2 = now_ns();
        int64_t delivered = 0;
        for (Req *r : done) delivered += r->n_result;
        {
            std::lock_guard<std::mutex> lk(mu);
            const int64_t t = now_ns();
            for (Req *r : done) {
                r->t_done = t;
                r->done = true;
            }
            st.requests += (int64_t)done.size();
            st.bytes += bytes;
            st.matches += delivered;
            st.deliver_ns += (t1 - t0) + (t - t2);
        }
        cv_done.notify_all();
        return PFSM_OK;
    }

    // Take queued requests for a batch (FIFO) while they fit the budget.
    bool admit(Slot &sl) {
        std::lock_guard<std::mutex> lk(mu);
        if (queue.empty()) return false;
        int64_t bytes = 0, rows = 0;
        while (!queue.empty() && (int32_t)sl.reqs.size() < max_batch) {
            Req *r = queue.front();
            const int64_t n = r->n;
            if (!sl.reqs.empty() && bytes + n > kBatchBytes) break;
            const int64_t est = out_estimate(r);
            const int64_t add = charge(bytes + n, rows + est) - charge(bytes, rows);
            // the first request of a batch is admitted when nothing else is in
            // flight, so a request larger than the budget still runs
            const bool first_alone = sl.reqs.empty() && inflight == 0;
            if (!first_alone && inflight + charge(bytes, rows) + add > budget) break;
            queue.pop_front();
            sl.reqs.push_back(r);
            bytes += n;
            rows += est;
        }
        if (sl.reqs.empty()) return false;
        sl.bytes = bytes;
        sl.out_cap = rows;
        inflight += charge(bytes, rows);
        st.peak_inflight = std::max(st.peak_inflight, inflight);
        return true;
    }

    void loop() {
        (void)hipSetDevice(device);
        for (;;) {
            bool progress = false;
            for (Slot &sl : slots) {
                if (!sl.busy || hipEventQuery(sl.ev) != hipSuccess) continue;
                const int rc = complete(sl);
                if (rc) finish(sl, rc);
                progress = true;
            }
            for (Slot &sl : slots) {
                if (sl.busy) continue;
                if (!admit(sl)) break;
                sl.busy = true;
                const int rc = launch(sl);
                if (rc) finish(sl, rc);
                progress = true;
            }
            if (progress) continue;
            bool any_busy = false;
            for (Slot &sl : slots) any_busy |= sl.busy;
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && !any_busy) return;
            if (any_busy) {
                // a batch is on the device: poll it, waking early for new work
                cv_work.wait_for(lk, std::chrono::microseconds(20));
            } else {
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            }
        }
    }
};

extern "C" {

int pfsm_server_create(pfsm_server_t **out, pfsm_t *const *hs, int32_t n_automata, int64_t mem_budget,
                       int32_t max_batch) {
    if (!out || !hs) return fail(PFSM_EINVAL, "NULL argument");
    if (n_automata < 1 || n_automata > kMaxBatchAutomata)
        return fail(PFSM_EINVAL, "n_automata must be in [1, %d]", kMaxBatchAutomata);
    for (int a = 0; a < n_automata; ++a)
        if (!hs[a]) return fail(PFSM_EINVAL, "handle %d is NULL", a);
    if (mem_budget < 1 || max_batch < 1) return fail(PFSM_EINVAL, "mem_budget and max_batch must be >= 1");
    std::unique_ptr<pfsm_server> sv(new (std::nothrow) pfsm_server);
    if (!sv) return fail(PFSM_ENOMEM, "server");
    sv->hs.assign(hs, hs + n_automata);
    sv->density.assign(n_automata, 1.0 / 16);
    sv->pool = std::make_unique<CopyPool>(kCopyThreads);
    sv->budget = mem_budget;
    sv->max_batch = max_batch;
    HIP_TRY(hipGetDevice(&sv->device));
    for (Slot &sl : sv->slots) {
        HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&sl.kdone, hipEventDisableTiming));
    }
    pfsm_server *p = sv.get();
    sv->worker = std::thread([p] { p->loop(); });
    *out = sv.release();
    return PFSM_OK;
}

static int server_submit(pfsm_server_t *sv, int32_t automaton, const uint8_t *bytes, int64_t n, int64_t *id,
                         bool copy) {
    if (!sv || !id || (n > 0 && !bytes)) return fail(PFSM_EINVAL, "NULL argument");
    if (automaton < 0 || automaton >= (int32_t)sv->hs.size())
        return fail(PFSM_EINVAL, "automaton %d outside [0, %d)", automaton, (int)sv->hs.size());
    if (n < 0 || n > kMaxStream) return fail(PFSM_EINVAL, "n must be in [0, 2^31 - 16]");
    auto r = std::make_unique<Req>();
    r->t_submit = now_ns();
    r->aut = automaton;
    r->n = n;
    if (copy) {
        r->bytes.assign(bytes, bytes + n);
        r->src = r->bytes.data();
    } else {
        r->src = bytes;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return fail(PFSM_EINVAL, "server is shutting down");
        r->id = sv->next_id++;
        *id = r->id;
        sv->queue.push_back(r.get());
        sv->reqs.emplace(r->id, std::move(r));
    }
    sv->cv_work.notify_one();
    return PFSM_OK;
}

int pfsm_server_submit(pfsm_server_t *sv, int32_t automaton, const uint8_t *bytes, int64_t n, int64_t *id) {
    return server_submit(sv, automaton, bytes, n, id, true);
}

int pfsm_server_submit_borrowed(pfsm_server_t *sv, int32_t automaton, const uint8_t *bytes, int64_t n,
                                int64_t *id) {
    return server_submit(sv, automaton, bytes, n, id, false);
}

int pfsm_server_wait(pfsm_server_t *sv, int64_t id, const pfsm_match_t **matches, int64_t *n_matches) {
    if (!sv || !matches || !n_matches) return fail(PFSM_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(PFSM_ENOENT, "no request %lld", (long long)id);
    Req *r = it->second.get();
    sv->cv_done.wait(lk, [&] { return r->done; });
    if (r->status != PFSM_OK) return fail(r->status, "request %lld failed", (long long)id);
    *matches = r->result;
    *n_matches = r->n_result;
    return PFSM_OK;
}

int pfsm_server_times(pfsm_server_t *sv, int64_t id, int64_t *t_submit_ns, int64_t *t_done_ns) {
    if (!sv || !t_submit_ns || !t_done_ns) return fail(PFSM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(PFSM_ENOENT, "no request %lld", (long long)id);
    *t_submit_ns = it->second->t_submit;
    *t_done_ns = it->second->done ? it->second->t_done : 0;
    return PFSM_OK;
}

int pfsm_server_release(pfsm_server_t *sv, int64_t id) {
    if (!sv) return fail(PFSM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(PFSM_ENOENT, "no request %lld", (long long)id);
    if (!it->second->done) return fail(PFSM_EINVAL, "request %lld is not finished", (long long)id);
    sv->reqs.erase(it);
    return PFSM_OK;
}

int pfsm_server_stats_get(pfsm_server_t *sv, pfsm_server_stats *out) {
    if (!sv || !out) return fail(PFSM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    return PFSM_OK;
}

void pfsm_server_destroy(pfsm_server_t *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (Slot &sl : sv->slots) sl.release();
    delete sv;
}

}  // extern "C"
