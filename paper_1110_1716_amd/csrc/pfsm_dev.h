// Device-side layouts shared by the host library and the HIP kernels of
// libpfsm.  Nothing here is part of the public ABI (include/pfsm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfsmk {

// Per-state flag bits (a byte per state).
constexpr uint8_t kLive = 1;   // some final state with an enabled label is reachable
constexpr uint8_t kFinal = 2;  // the state carries at least one enabled label

// Cross-workgroup count slot of the NFA's persistent grid: a 24-bit epoch
// over a 40-bit count.  Every workgroup rewrites its slot once per round, so
// all slots carry the same epoch when a launch begins; a workgroup reads its
// own slot's epoch, adds one, and waits for its peers to reach it.
constexpr int kEpochShift = 40;
constexpr unsigned long long kCountMask = (1ull << kEpochShift) - 1;
constexpr unsigned kEpochMask = (1u << 24) - 1;

// Scan control block of a workspace (device memory, zeroed once).  Segments
// are handed out in order by `ticket`; `done` counts the workgroups that have
// finished, and the last one resets both and advances `epoch`, so successive
// launches (or replays of a captured launch) need no host bookkeeping.
struct ScanCtl {
    unsigned long long ticket;
    unsigned epoch;
    unsigned done;
};

// Look-back word of a segment: epoch (22 bits) | status (2 bits) | value
// (40 bits, saturating).  Status 1: the value is the segment's own count;
// status 2: the value is the count up to and including the segment.
constexpr int kLbStatShift = 40;
constexpr int kLbEpochShift = 42;
constexpr unsigned long long kLbValMask = (1ull << 40) - 1;
constexpr unsigned kLbEpochMod = (1u << 22) - 1;  // epochs in use: 1 .. kLbEpochMod
constexpr int kLbAgg = 1, kLbIncl = 2;

// Segments of a batch launch (stream_off == nullptr: one stream, x[0, n)).
// x holds every stream; the launch's segments, their streams and the output
// base are written on the device by the planning kernels.
struct SegPlan {
    const int64_t *stream_off;  // [n_streams + 1] byte offsets into x
    const int32_t *seg_stream;  // stream of each segment, from *seg_base_dev on
    const int32_t *seg_first;   // [n_streams] first segment of each stream in its launch
    const int32_t *n_segs_dev;  // segments of this launch
    const int32_t *seg_base_dev;
    const int64_t *base_dev;    // output index of this launch's first match
    const int64_t *seg_dev;     // bytes per segment of this launch
    int64_t *stream_lo;         // [n_streams] each stream's range in the output
    int64_t *stream_hi;
};

struct MatchOut {
    int32_t start, end, label;
};

// Instances still live when a scan reaches the end of its input (chained
// partitioning, Section III.D.2): each appends one (start, state) pair per
// state it holds, start as a position of the whole stream (the piece's
// first byte is `base`).  Pairs arrive in no particular order and may repeat;
// *n counts every pair asked for, including those past cap.  Off when pairs
// is null.
struct CarryOut {
    uint32_t *pairs;          // [2 * cap]
    unsigned long long *n;
    int64_t cap;
    int32_t base;
    int32_t pad;
};

__device__ __forceinline__ unsigned long long carry_reserve(const CarryOut &c, int cnt) {
    return atomicAdd(c.n, (unsigned long long)cnt);
}

// Pair `slot` of a reservation: the instance started at `start` (a position
// of the piece) holds `state`.
__device__ __forceinline__ void carry_write(const CarryOut &c, unsigned long long slot, int32_t start,
                                            uint32_t state) {
    if (slot < (unsigned long long)c.cap) {
        c.pairs[2 * slot] = (uint32_t)(c.base + start);
        c.pairs[2 * slot + 1] = state;
    }
}

// ---------------------------------------------------------------- DFA scan

constexpr int kDfaThreads = 768;               // one workgroup, 12 wave64
constexpr int kDfaWaves = kDfaThreads / 64;
constexpr int kDfaWin = 1024;                  // bytes per wave window, 16 per lane
constexpr int kDfaRing = 2 * kDfaWin;          // staged bytes per wave: window and the next
constexpr int kDfaSegMax = 65536;              // bytes per workgroup and round
constexpr int kDfaQueue = 128;                 // LDS queue entries per wave
constexpr int kDfaList = kDfaWin / 2;          // live-start list per wave (half a window), 32-bit entries
constexpr int kDfaMatchCap = 1024;             // LDS match buffer per workgroup
constexpr int kDfaSpill = 4096;                // walks a workgroup can park in memory per segment
constexpr int kDfaLdsLimit = 159 * 1024;       // dynamic LDS: 160 KiB per CU less the static variables
constexpr int kDfaTableBudget = 96 * 1024;     // resident table bytes
// Flag bytes kept in LDS for kEnc8: entries from n_states on are zero, so
// the "no transition" value 255 reads as not live.
constexpr int kDfaFlags8 = 256;
constexpr int kDfaHotBudget = 48 * 1024;       // cached rows when not resident

// How the transition table is read.  Resident encodings keep the whole
// table, the state flags and the label CSR in LDS; the cold ones read them
// through L2 (rows of q0's successors are still copied to LDS).  Every
// encoding decodes to the given values.
enum DfaEnc : int {
    kEnc8 = 0,    // n_states <= 255: uint8, 255 stands for -1
    kEnc8D = 1,   // n_states == 256: uint8 low byte + one "no transition" bit
    kEnc16 = 2,   // n_states <= 32767: int16
    kCold16 = 3,  // int16 in HBM/L2
    kCold32 = 4,  // int32 in HBM/L2
};

struct DfaArgs {
    const uint8_t *x;           // 16-byte aligned
    int64_t n;
    const void *tbl;            // table as stored in HBM (int16 or int32)
    const void *res;            // LDS image from off_flags on: flags, label CSR, table (or cached rows)
    int32_t res_bytes;
    int32_t n_states, n_symbols;
    const int16_t *b2s;         // [256] byte -> symbol, -1 = not in the alphabet
    const int32_t *first;       // [256] live target of q0 on each byte, else -1
    const int16_t *first_slot;  // [256] row slot of first[b] in the cached rows, -1 = none
    const void *hot;            // cold encodings: [n_hot * n_symbols] cached rows
    int32_t n_hot;
    const uint8_t *flags;       // [n_states] kLive | kFinal
    const int32_t *lab_off;     // [n_states + 1]
    const int32_t *lab;         // enabled labels, sorted and unique per state
    MatchOut *out;
    int64_t cap;
    int64_t *total;             // grand total (device)
    ScanCtl *ctl;
    unsigned long long *lb;     // [lb_cap] look-back words, one per segment
    int32_t lb_cap;
    int32_t n_segs;             // segments of this launch (single stream)
    SegPlan plan;               // batches
    long long *bstats;          // [gridDim.x * 4] T, X, long walks, matches
    void *spill;                // [gridDim.x * kDfaSpill] walks parked out of LDS
    int64_t seg;                // bytes per segment (multiple of 16)
    CarryOut carry;             // live instances at the end of the input
    // dynamic LDS layout, byte offsets
    int32_t off_flags, off_laboff, off_lab, off_tab, off_q, off_m, off_list, lds_bytes;
};

// Fixed LDS head: wave rings, hot-row slot by byte, byte map, q0's live
// target by byte as 16-bit words (bit 15: live, bits 0-14: the state).
constexpr int kDfaLdsFixed = kDfaWaves * kDfaRing + 256 * 2 + 256 * 2 + 256 * 2;

// Tag-merged DFA scan: one wave per segment of kMergedSeg starts, for
// automata with at most kMergedStates states (one entry per lane).
constexpr int kMergedThreads = 256;
constexpr int kMergedSeg = 1024;
constexpr int kMergedStates = 63;

// Dynamic LDS of the tag-merged scan: its byte-indexed table.
inline size_t merged_lds(int n_states) { return ((size_t)n_states * 256 + 15) / 16 * 16; }

struct MergedArgs {
    const uint8_t *x;           // any alignment
    int64_t n;
    const uint8_t *tab;         // [n_states * 256] by byte: live target | 128 when final, 255 = none
    const int32_t *lab_off;     // [n_states + 1]
    const int32_t *lab;
    int32_t n_states, q0;
    MatchOut *out;
    int64_t cap;
    int64_t *total;
    ScanCtl *ctl;               // segment tickets
    unsigned long long *lb;     // look-back words (reset by the last workgroup; unused otherwise)
    int32_t lb_cap, n_segs;
    long long *bstats;          // [gridDim.x * 4] (count launch)
    long long *tag_cnt;         // [n] matches of each start (count launch writes, write launch reads)
    long long *seg_cnt;         // [n_segs] matches of each segment
    long long *seg_base;        // [n_segs + 1] their exclusive scan
    int32_t pass;               // 0: count launch, 1: write launch
    int32_t narrow_max;         // largest per-start count or segment offset kept in 32-bit LDS words
};

// Host-side kernel handles (defined in the .hip translation units).
const void *dfa_kernel_fn(int enc, bool identity_map);
hipError_t launch_dfa_merged(const MergedArgs &a, int grid, hipStream_t s);
const void *dfa_merged_fn();
hipError_t launch_write_zero(int64_t *p, hipStream_t stream);

}  // namespace pfsmk

// ---------------------------------------------------------------- NFA scan

namespace pfsmk {

constexpr int kNfaThreads = 256;             // workgroup: 4 wave64
constexpr int kNfaWindow = kNfaThreads * 16; // 16 starts per thread
constexpr int kNfaSegMax = 65536;            // bytes per workgroup and round
constexpr int kNfaK = 4;                     // states a queued walk keeps in registers
constexpr int kNfaQueue = 64;                // walk queue entries per wave
constexpr int kNfaMatchCap = 1024;           // LDS match buffer per workgroup
constexpr int kNfaBigCap = 256;              // replayed starts listed per workgroup
constexpr int kNfaGapCap = 192;              // gap walks waiting for a gap pass, per wave
constexpr int kNfaLabelsMax = 1 << 24;       // labels per state

// Packed state record, one 32-byte load per state and step.  Only live
// targets are kept (a state is live when a final state with an enabled label
// is reachable from it): the instance drops the others at once anyway.
//   info: bit 0 live, bit 1 final, bit 2 edges inline, bits 8.. label count
//   edge test word: bits 0-7 byte, bits 8-9 kind (0 one byte, 1 any byte,
//     2 class bitmap), bits 10-31 class id
//   edge target word: bit 31 clear: a state whose epsilon closure is itself,
//     bit 31 set: index of its closure list; bit 30: the state is final
struct __attribute__((aligned(16))) NfaRec {
    uint32_t info;
    int32_t lab_off;
    int32_t edge_off;  // into the edge array when not inline
    int32_t n_edges;
    uint32_t e0_test, e0_tgt, e1_test, e1_tgt;
};
constexpr uint32_t kRecLive = 1, kRecFinal = 2, kRecInline = 4, kRecGap = 8, kRecGapFin = 16;
// A gap state (kRecGap) is a state of a bounded any-byte gap: state q with
// exactly two inline edges, e0 = an edge E and e1 = any byte to q + 1, where
// q + 1 carries the same E and either continues the gap the same way or
// ends it with E alone.  edge_off holds how many any-byte steps remain
// (at least 1).  A walk whose whole set is one gap state can pass every byte
// that E rejects, up to that many, without reading records: each such byte
// moves it to the next state of the gap.
// kRecGapFin marks a gap state whose E leads into a simple chain (one edge
// per state, the last state alone final and without edges).  Its lab_off
// holds the test of the chain's first edge (0 when E's target is the end).

// The lists of a byte pair in the pair cache: p_st[st_lo, st_hi) and
// p_lab[lab_lo, lab_hi); one 16-byte load.
struct __attribute__((aligned(16))) PairRange {
    int32_t st_lo, st_hi, lab_lo, lab_hi;
};
constexpr uint32_t kTgtList = 1u << 31, kTgtFinal = 1u << 30, kStateMask = (1u << 30) - 1;

struct NfaArgs {
    const uint8_t *x;  // 16-byte aligned
    int64_t n;
    int32_t n_states;           // state capacity of the tables: the replay scratch stride
    const NfaRec *rec;          // [n_states]
    const uint32_t *edges;      // (test, target) pairs for records with more than two edges
    const uint32_t *class_bits; // [n_classes * 8]
    const int32_t *cl_off;      // closure lists: [n_lists + 1]
    const uint32_t *cl;         // target words
    const int32_t *lab;         // enabled labels, sorted and unique per state
    // first symbol: closure(delta(closure({q0}), c)) restricted to live states
    const int32_t *f1_off;      // [257]
    const uint32_t *f1;         // target words
    const int32_t *e1_off;      // [257] labels reported after the first symbol
    const int32_t *e1;
    // first two symbols (when pair_on): the same for the byte pair (c1, c2)
    int32_t pair_on;
    const uint32_t *p_bits;     // [2048] pair has states or labels
    const PairRange *p_rng;     // [65536] where each pair's lists lie
    const uint32_t *p_st;       // target words
    const int32_t *p_lab;
    MatchOut *out;
    int64_t cap;
    int64_t *total;
    ScanCtl *ctl;
    unsigned long long *lb;     // [lb_cap] look-back words, one per segment
    int32_t lb_cap;
    int32_t n_segs;
    SegPlan plan;
    long long *bstats;          // [gridDim.x * 4]
    int64_t seg;
    // per-workgroup replay scratch: two frontiers of n_states entries and a
    // bitset of n_states bits (all clear between uses); state ids are below
    // n_states
    uint32_t *big_front;        // [gridDim.x * 2 * n_states]
    uint32_t *big_bits;         // [gridDim.x * ((n_states + 31) / 32)]
    CarryOut carry;             // live instances at the end of the input
};

// The scan kernel; `carry`: the variant that collects live instances at the
// end of its input.
const void *nfa_kernel_fn(bool carry);

}  // namespace pfsmk
