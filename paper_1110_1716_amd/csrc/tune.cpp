// Autotuner over a handle's launch settings: tag-merged stepping (small
// DFAs), the bytes per segment (the window a workgroup takes per ticket),
// resident workgroups per compute unit, and the LDS budget of the read-only
// caches (a DFA's transition table resident in LDS or read through L2 with
// hot rows cached; an NFA's two-symbol cache on or off).  The number of
// starts per lane and of states a lane keeps per walk are fixed when the
// kernels are compiled.
//
// Settings are tried one knob at a time, each on a scan of a caller's
// sample timed with HIP events, and a change is kept when it saves at least
// 2 %.  Every setting must reproduce the match list of the first one, entry
// by entry: knobs change where work runs, never what is found.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "host_common.h"
#include "pfsm.h"

using namespace pfsmk;

namespace {

struct Timer {
    pfsm_t *h;
    const uint8_t *x;
    int64_t n;
    int32_t reps;
    int64_t count;
    pfsm_match_t *out;
    int64_t *d_cnt;
    hipStream_t s;
    hipEvent_t e0, e1;
    int tried = 0;
    std::vector<pfsm_match_t> ref, cur;  // the first setting's list, the latest one

    // Mean time per scan (ms) under the handle's current settings.
    int time(double *ms) {
        int rc = pfsm_scan_async(h, x, n, out, count, d_cnt, s);  // warm-up, grows buffers
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r)
            if ((rc = pfsm_scan_async(h, x, n, out, count, d_cnt, s))) return rc;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        int64_t got = -1;
        HIP_TRY(hipMemcpy(&got, d_cnt, sizeof got, hipMemcpyDeviceToHost));
        if (got != count)
            return fail(PFSM_EINVAL, "a tuning setting changed the match count (%lld, expected %lld)", (long long)got,
                        (long long)count);
        std::vector<pfsm_match_t> &dst = tried == 0 ? ref : cur;
        dst.resize((size_t)count);
        if (count > 0) HIP_TRY(hipMemcpy(dst.data(), out, sizeof(pfsm_match_t) * (size_t)count, hipMemcpyDeviceToHost));
        if (tried > 0 && count > 0 && std::memcmp(ref.data(), dst.data(), sizeof(pfsm_match_t) * (size_t)count) != 0)
            return fail(PFSM_EINVAL, "a tuning setting changed the match list");
        *ms = (double)t / reps;
        ++tried;
        return PFSM_OK;
    }
};

}  // namespace

extern "C" {

int pfsm_tune(pfsm_t *h, const uint8_t *d_sample, int64_t n, int32_t reps, pfsm_tune_report *report,
              void *hip_stream) {
    if (!h || !d_sample || !report) return fail(PFSM_EINVAL, "NULL argument");
    if (n <= 0 || n > kMaxStream) return fail(PFSM_EINVAL, "sample size must be in [1, 2^31 - 16]");
    if (reps < 1 || reps > 10000) return fail(PFSM_EINVAL, "reps must be in [1, 10000]");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int64_t v = 0;
    const bool dfa = pfsm_get_option(h, PFSM_OPT_TABLE_BUDGET, &v) == PFSM_OK;
    const int cache_opt = dfa ? PFSM_OPT_TABLE_BUDGET : PFSM_OPT_PAIR_CACHE;

    Timer tm{h, d_sample, n, reps, 0, nullptr, nullptr, s, nullptr, nullptr};
    int rc = pfsm_scan(h, d_sample, n, nullptr, 0, &tm.count, hip_stream);
    if (rc != PFSM_OK && rc != PFSM_EOVERFLOW) return rc;
    HIP_TRY(hipMalloc(&tm.out, sizeof(pfsm_match_t) * (size_t)(tm.count > 0 ? tm.count : 1)));
    HIP_TRY(hipMalloc(&tm.d_cnt, sizeof(int64_t)));
    HIP_TRY(hipEventCreate(&tm.e0));
    HIP_TRY(hipEventCreate(&tm.e1));

    double before = 0, best = 0;
    auto tune_knob = [&](int opt, const std::vector<int64_t> &cands) -> int {
        int64_t keep = 0;
        int r = pfsm_get_option(h, opt, &keep);
        if (r) return r;
        for (int64_t c : cands) {
            if (c == keep) continue;
            if ((r = pfsm_set_option(h, opt, c, hip_stream))) return r;
            double ms = 0;
            if ((r = tm.time(&ms))) return r;
            if (ms < best * 0.98) {
                best = ms;
                keep = c;
            }
        }
        return pfsm_set_option(h, opt, keep, hip_stream);
    };

    if (!(rc = tm.time(&before))) {
        best = before;
        // 0. tag-merged stepping, where the automaton allows it
        if (dfa) {
            int64_t cur = 0;
            pfsm_get_option(h, PFSM_OPT_MERGED_WALKS, &cur);
            if (pfsm_set_option(h, PFSM_OPT_MERGED_WALKS, 1, hip_stream) == PFSM_OK &&
                !(rc = pfsm_set_option(h, PFSM_OPT_MERGED_WALKS, cur, hip_stream)))
                rc = tune_knob(PFSM_OPT_MERGED_WALKS, {0, 1});
        }
        int64_t merged = 0;
        if (dfa) pfsm_get_option(h, PFSM_OPT_MERGED_WALKS, &merged);
        // 1. LDS budget of the caches (the merged scan has its own table)
        if (!rc && dfa) {
            int64_t resident = 0;
            pfsm_get_option(h, PFSM_OPT_RESIDENT_TABLE, &resident);
            if (resident && !merged) rc = tune_knob(PFSM_OPT_TABLE_BUDGET, {-1, 0});
        } else if (!rc) {
            rc = tune_knob(PFSM_OPT_PAIR_CACHE, {1, 0});
        }
        // 2. resident workgroups per compute unit
        if (!rc) {
            int64_t occ = 1;
            pfsm_get_option(h, PFSM_OPT_MAX_WORKGROUPS_PER_CU, &occ);
            std::vector<int64_t> c{0};
            for (int64_t k = 1; k < occ; ++k) c.push_back(k);
            rc = tune_knob(PFSM_OPT_WORKGROUPS_PER_CU, c);
        }
        // 3. bytes per segment (fixed in the merged scan)
        if (!rc && !merged) rc = tune_knob(PFSM_OPT_SEGMENT, {0, 4096, 8192, 16384, 32768, 65536});
    }
    (void)hipEventDestroy(tm.e0);
    (void)hipEventDestroy(tm.e1);
    (void)hipFree(tm.out);
    (void)hipFree(tm.d_cnt);
    if (rc) return rc;
    pfsm_get_option(h, PFSM_OPT_SEGMENT, &report->segment);
    pfsm_get_option(h, PFSM_OPT_WORKGROUPS_PER_CU, &report->workgroups_per_cu);
    report->table_budget = -1;
    report->pair_cache = -1;
    pfsm_get_option(h, cache_opt, dfa ? &report->table_budget : &report->pair_cache);
    report->ms_before = before;
    report->ms_after = best;
    report->configs = tm.tried;
    report->matches = tm.count;
    report->merged_walks = 0;
    if (dfa) pfsm_get_option(h, PFSM_OPT_MERGED_WALKS, &report->merged_walks);
    return PFSM_OK;
}

}  // extern "C"
