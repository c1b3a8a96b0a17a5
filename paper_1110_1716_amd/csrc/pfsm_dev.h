// Device-side layouts shared by the host library and the HIP kernels of
// libpfsm.  Nothing here is part of the public ABI (include/pfsm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfsmk {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kOverlap = 256;      // bytes staged past a window's end
constexpr int kFlagsLds = 8192;    // state flags cached in LDS up to this many states

// Per-state flag bits (a byte per state).
constexpr uint8_t kLive = 1;   // some final state with an enabled label is reachable
constexpr uint8_t kFinal = 2;  // the state carries at least one enabled label

// Decoupled look-back status word: 2 flag bits over a 62-bit count.
constexpr unsigned long long kStatAgg = 1ull << 62;
constexpr unsigned long long kStatPre = 2ull << 62;
constexpr unsigned long long kStatVal = (1ull << 62) - 1;

// Control block of one scan workspace.  ticket/done return to zero at the
// end of every launch (the last workgroup to finish resets them and the
// status words), so consecutive launches on one stream need no memset.
struct ScanCtl {
    unsigned int ticket;
    unsigned int done;
    unsigned long long acc[4];  // running T, X, long walks, matches
    long long last[4];          // the previous launch's totals
};

struct MatchOut {
    int32_t start, end, label;
};

// DFA scan arguments.
struct DfaArgs {
    const uint8_t *x;
    int64_t n;
    const void *tbl;          // int16 or int32 [n_states * n_symbols], as given
    int32_t n_states, n_symbols;
    const int16_t *b2s;       // [256] byte -> symbol, -1 = not in the alphabet
    const int32_t *first;     // [256] live target of q0 on each byte, else -1
    const uint8_t *flags;     // [n_states] kLive | kFinal
    const int32_t *lab_off;   // [n_states + 1]
    const int32_t *lab;       // enabled labels, sorted and unique per state
    MatchOut *out;
    int64_t cap;
    int64_t *total;           // grand total (device)
    ScanCtl *ctl;
    unsigned long long *status;  // [n_windows]
    int32_t n_windows;
};

// Host-side launchers (defined in the .hip translation units).
hipError_t launch_dfa_scan(const DfaArgs &a, int per_thread, bool identity_map, bool tbl16,
                           hipStream_t stream);
hipError_t launch_write_zero(int64_t *p, hipStream_t stream);

}  // namespace pfsmk
