// Streaming scans (chained partitioning, Section III.D.2): argument blocks
// of the kernels that carry live instances from one piece of a stream to the
// next (internal to libpfsm).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfsm_dev.h"

namespace pfsmk {

// Instances carried into a piece: keys (start << 32 | state), sorted and
// unique; instance g (one start) holds keys [grp_off[g], grp_off[g + 1]).  A
// DFA instance has one state, an NFA instance a set.  Counts live on the
// device so that no host round trip sits between the kernels of a piece.
struct CarrySet {
    const unsigned long long *keys;
    const int32_t *grp_off;  // [n_groups + 1]
    const int32_t *n_groups;
};

// Advance every carried DFA instance through the piece x[0, n).  Count pass
// (write == 0): cnt[g] = its matches; instances still live after x go to
// `carry`.  Write pass: its matches from out[off[g]] on, in (end, label)
// order.  The table is the one given at load (int16 or int32, n_symbols
// columns; bytes map to columns through b2s unless identity).
struct DfaResumeArgs {
    const uint8_t *x;
    int64_t n;
    int32_t base;  // stream position of x[0]
    int32_t tbl16, n_symbols, identity;
    const void *tbl;
    const int16_t *b2s;
    const uint8_t *flags;
    const int32_t *lab_off;
    const int32_t *lab;
    CarrySet in;
    int64_t *cnt;
    const int64_t *off;
    MatchOut *out;
    int64_t cap;
    CarryOut carry;
    int32_t write;
};

// The same for NFA instances, one workgroup per instance with its frontier
// in the workgroup's replay scratch (a.big_front, a.big_bits); a.x and a.n
// are the piece, a.carry receives the instances still live after it.
struct NfaResumeArgs {
    NfaArgs a;
    int32_t base;
    int32_t write;
    CarrySet in;
    int64_t *cnt;
    const int64_t *off;
};

hipError_t launch_dfa_resume(const DfaResumeArgs &r, hipStream_t s);
hipError_t launch_nfa_resume(const NfaResumeArgs &r, int grid, hipStream_t s);

}  // namespace pfsmk
