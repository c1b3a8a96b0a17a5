// NFA half of the host library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>

#include "host_common.h"
#include "pfsm.h"
#include "pfsm_dev.h"
#include "stream.h"

namespace pfsmk {

struct NfaHost;
struct NfaDeleter {
    void operator()(NfaHost *p) const;
};
using NfaPtr = std::unique_ptr<NfaHost, NfaDeleter>;

int nfa_load(const pfsm_nfa_desc *d, hipStream_t s, NfaPtr *out);
int nfa_add_pattern(NfaHost *h, const pfsm_nfa_desc *p, hipStream_t s);
int nfa_remove_pattern(NfaHost *h, int32_t label, hipStream_t s);
int nfa_scan_async(NfaHost *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap, int64_t *d_total,
                   hipStream_t s);
// One launch of the scan kernel: a single stream (plan == nullptr) or the
// segments of a batch plan.
// d_base (single stream only): output index of the first match, on the
// device; carry: collects the instances still live at the end of x.
int nfa_launch(NfaHost *h, const uint8_t *x, int64_t n, const SegPlan *plan, int64_t seg, MatchOut *out,
               int64_t cap, int64_t *d_total, hipStream_t s, const int64_t *d_base = nullptr,
               const CarryOut *carry = nullptr);
// Count (write == 0) or write pass over carried instances (stream.h).
int nfa_resume(NfaHost *h, const uint8_t *x, int64_t n, int32_t base, const CarrySet &in, int64_t *cnt,
               const int64_t *off, MatchOut *out, int64_t cap, const CarryOut &carry, int write, hipStream_t s);
int nfa_grid_blocks(NfaHost *h);
Knobs *nfa_knobs(NfaHost *h);
int nfa_occupancy(NfaHost *h);
// Advances whenever an edit or option moves the handle's device tables or
// changes a scalar its launches carry.
uint64_t nfa_layout_epoch(NfaHost *h);
// After a change of h's knobs: the grid, and the tables when `tables`.
int nfa_apply_knobs(NfaHost *h, bool tables, hipStream_t s);
WorkspacePool *nfa_pool(NfaHost *h);

}  // namespace pfsmk
