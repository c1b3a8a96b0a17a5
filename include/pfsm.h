/*
 * pfsm.h -- C ABI of libpfsm, an all-matches Parallel Finite State Machine
 * scanner for AMD Instinct MI355X (gfx950).
 *
 * A PFSM (Section III.A) is the tuple (Sigma, Q, q0, delta, F, L, l): an
 * automaton whose transition function may be deterministic or not, whose
 * final states carry labels naming the regular expression they accept, and
 * which is run with a fresh instance started at every input position
 * (Section III.B).  A scan reports every match as a triple
 * (start, end, label): the instance started at `start` entered, after
 * consuming input[end], a final state labelled `label` (Section III.B,
 * reporting rule; Fig. 2 lists such triples).  Overlapping and nested
 * matches are all reported.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Positions are 0-based, `end` is inclusive, 0 <= start <= end < n.
 *   Empty matches are never reported: a match consumes at least one byte.
 * - The match set is a set: each (start, end, label) appears once, even when
 *   several final states carrying the same label are entered at once.
 * - Output order is ascending (start, end, label).
 * - Labels are int32 >= 0.  A final state may carry several labels (a label
 *   set); a state with an empty label set is not final.
 * - Every call returns PFSM_OK (0) or a negative PFSM_E* code and never
 *   throws across the ABI.  pfsm_last_error() returns a description of the
 *   calling thread's most recent failure.
 * - Streams: every `hip_stream` argument is a hipStream_t (NULL = the null
 *   stream).  All device work of a call is ordered on that stream.
 * - Ownership: the library copies every host descriptor array during the
 *   call; the caller keeps ownership of them.  Device input and output
 *   buffers belong to the caller and are never freed by the library.  The
 *   handle owns its device tables and per-stream scan workspaces until
 *   pfsm_free().
 * - Threads: one handle must not be mutated (add/remove/free) concurrently
 *   with any other call on it.  Scans on one handle issued on different
 *   streams may overlap; scans on the same stream run in stream order.
 */
#ifndef PFSM_H
#define PFSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfsm pfsm_t;

/* One match: 0-based positions, end inclusive (Fig. 2 prints [start-end]). */
typedef struct {
    int32_t start, end, label;
} pfsm_match_t;

/* A DFA (Section II: (Sigma, Q, q0, delta, F)) with labelled final states
 * (Section III.A: L and l).
 *   n_states        |Q|, >= 1; q0 in [0, n_states).
 *   n_symbols       |Sigma|, >= 1, n_states * n_symbols < 2^31.
 *   byte_to_symbol  [256] host array: symbol of each input byte, or -1 when
 *                   the byte is not in Sigma (an instance reading it ends).
 *                   NULL means the identity map and requires n_symbols == 256.
 *   delta           [n_states * n_symbols] host array, row-major
 *                   (delta[q * n_symbols + s]); a target state or -1 for "no
 *                   transition" (the instance ends).  Used as given.
 *   final_off       [n_states + 1] host array, CSR offsets into final_labels;
 *                   final_off[0] == 0, non-decreasing.
 *   final_labels    [final_off[n_states]] host array: the label set of each
 *                   state (duplicates allowed, reported once).            */
typedef struct {
    int32_t n_states, n_symbols, q0;
    const int16_t *byte_to_symbol;
    const int32_t *delta;
    const int32_t *final_off, *final_labels;
} pfsm_dfa_desc;

/* An NFA (Section II: delta: Q x Sigma -> P(Q)) with epsilon edges and
 * labelled final states, as CSR successor lists over byte classes.
 *   n_states        |Q| >= 1; q0 in [0, n_states).
 *   n_classes       number of byte classes (>= 0).
 *   row_ptr         [n_states + 1] CSR offsets; row_ptr[0] == 0.
 *   edge_class      [row_ptr[n_states]] class of each edge: -1 = epsilon,
 *                   k in [0, n_classes) = the byte set class_bits[k*8..k*8+7].
 *   edge_dst        [row_ptr[n_states]] target state of each edge.
 *   class_bits      [n_classes * 8] 256-bit byte sets: byte b is in class k
 *                   when bit (b % 32) of class_bits[k * 8 + b / 32] is set.
 *   final_off, final_labels  label sets, as for the DFA.
 * Epsilon edges taken right after a byte is consumed count for that byte's
 * position: a final state reached through them is reported with end = the
 * position of that byte.                                                   */
typedef struct {
    int32_t n_states, q0, n_classes;
    const int32_t *row_ptr, *edge_class, *edge_dst;
    const uint32_t *class_bits;
    const int32_t *final_off, *final_labels;
} pfsm_nfa_desc;

/* Work counters of the most recent scan on a stream (pfsm_last_stats).
 *   transitions  instance-steps: over all start positions, the number of
 *                bytes consumed while the instance had a live state (the
 *                byte that ends it included).  A state is live when some
 *                final state with an enabled label is reachable from it.
 *   activations  live states entered, summed over those steps.
 *   matches      the scan's match count.
 *   long_walks   instances that outlived their window's staged bytes.   */
typedef struct {
    int64_t transitions, activations, matches, long_walks;
} pfsm_stats;

enum {
    PFSM_OK = 0,
    PFSM_EINVAL = -1,    /* malformed descriptor or argument               */
    PFSM_ENOMEM = -2,    /* host or device allocation failed               */
    PFSM_EOVERFLOW = -3, /* more matches than `cap`; count still reported  */
    PFSM_EHIP = -4,      /* a HIP runtime call failed                      */
    PFSM_ENOENT = -5,    /* no pattern carries the label                   */
    PFSM_EEXIST = -6,    /* a pattern already carries the label            */
    PFSM_ENOSYS = -7     /* operation not supported for this handle kind   */
};

/* Load a DFA (Section II) as a PFSM.  The transition table is kept as given
 * (narrowed to 16-bit storage when n_states < 32768, values unchanged); the
 * library derives read-only caches from it (live flags, the row of q0 per
 * byte, label CSR).  On success *out owns the device copy.  Synchronises
 * `hip_stream` before returning.
 * Errors: PFSM_EINVAL (descriptor), PFSM_ENOMEM, PFSM_EHIP.               */
int pfsm_load_dfa(pfsm_t **out, const pfsm_dfa_desc *d, void *hip_stream);

/* Load an NFA (Section II/III.A) as a PFSM, for instance the union of
 * several expressions under an ancillary initial state with epsilon edges
 * (Section III.A).  No conversion to a DFA takes place.  Synchronises
 * `hip_stream` before returning.
 * Errors: PFSM_EINVAL, PFSM_ENOMEM, PFSM_EHIP.                            */
int pfsm_load_nfa(pfsm_t **out, const pfsm_nfa_desc *d, void *hip_stream);

/* Add an expression to a loaded NFA handle (Section III.A: expressions can
 * be added or removed efficiently; Section IV: with zero downtime).  The
 * pattern's automaton is put together with the handle's through an
 * ancillary initial state and an epsilon edge (Section III.A).  Its labels
 * must not occur in the handle.  The edit is incremental: only the new
 * pattern's tables are computed, the start tables are reassembled, and the
 * changed ranges are copied into the handle's device buffers in place.
 * Scans issued before the call keep the old automaton (the call waits for
 * them); scans issued after it (on any stream) see the new one.
 * HIP graphs: a graph that scans with this handle, captured while
 * PFSM_OPT_LAYOUT_EPOCH had some value, sees the edited automaton when it
 * is replayed after the edit as long as the epoch still has that value.
 * When an edit outgrows the buffers, the epoch advances: the old buffers
 * stay allocated (and unchanged) until pfsm_free, so such a graph still
 * replays safely, but it scans the automaton of its capture; capture it
 * again (after one pfsm_scan_batch on its stream, which sizes the stream's
 * workspace for the larger automaton).
 * Errors: PFSM_EINVAL, PFSM_EEXIST (label already present), PFSM_ENOSYS
 * (DFA handle: its table is monolithic), PFSM_ENOMEM, PFSM_EHIP.          */
int pfsm_add_pattern(pfsm_t *h, const pfsm_nfa_desc *pattern, void *hip_stream);

/* Remove an expression: after the call no match with `label` is reported.
 * Patterns added with pfsm_add_pattern are cut off the ancillary initial
 * state; otherwise the label is disabled in the label table, and only the
 * parts of the tables that lead to it are recomputed.  Tables only shrink,
 * so they are rewritten in place and PFSM_OPT_LAYOUT_EPOCH stays (for DFA
 * handles too).  Same snapshot and graph semantics as pfsm_add_pattern.
 * Errors: PFSM_ENOENT (label not present), PFSM_ENOMEM, PFSM_EHIP.        */
int pfsm_remove_pattern(pfsm_t *h, int32_t label, void *hip_stream);

/* Scan n bytes of device memory and report every match (Section III.B).
 *   d_input    device pointer to n bytes (any alignment); n in [0, 2^31 - 16].
 *   d_out      device array of `cap` pfsm_match_t, written in ascending
 *              (start, end, label) order.
 *   n_matches  host pointer, receives the total number of matches.
 * Returns PFSM_EOVERFLOW when the total exceeds cap: *n_matches is still
 * the exact total, d_out holds the first cap matches; retry with a larger
 * buffer.  Synchronises `hip_stream` (the only device-to-host crossing).  */
int pfsm_scan(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
              int64_t *n_matches, void *hip_stream);

/* pfsm_scan without the synchronisation: the total is written to the device
 * int64 `d_n_matches` in stream order, and only the first `cap` matches are
 * stored.  The caller compares *d_n_matches with cap once the stream has
 * reached it.  Errors are argument errors only (PFSM_EINVAL, PFSM_ENOMEM,
 * PFSM_EHIP).                                                             */
int pfsm_scan_async(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out,
                    int64_t cap, int64_t *d_n_matches, void *hip_stream);

/* pfsm_scan_async for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the call allocates nothing, neither device nor host memory.  Its scratch
 * (the scan's control block, look-back words, per-workgroup counters and
 * parked walks) is one static array of about 32.3 MiB in the library's
 * global memory, one copy per GPU, held until the process ends.  The first
 * call on a GPU clears the array's control words on `hip_stream`.
 *   Arguments, output and total as for pfsm_scan_async; DFA handles only.
 *   The scan uses at most 512 workgroups and 32768 segments: an input that
 *   the handle's segment size splits into more segments is rejected.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (concurrent streams, or host threads) race and must be serialised by
 * the caller.  pfsm_last_stats does not report these scans.
 * Errors: PFSM_EINVAL (arguments, or more than 32768 segments), PFSM_ENOSYS
 * (NFA handle), PFSM_EHIP.                                                 */
int pfsm_scan_noalloc(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
                      int64_t *d_n_matches, void *hip_stream);

/* Scan many byte streams, each against one of several handles, in one pass:
 * the union model of Section III.A applied per stream (each stream's
 * matches are those of pfsm_scan of its bytes alone against its handle).
 *   hs                  host array of n_automata handles.
 *   d_data              device bytes of all streams, concatenated.
 *   d_stream_off        device int64 [n_streams + 1]: stream i is
 *                       d_data[off[i], off[i+1]); each shorter than 2^31.
 *   d_stream_automaton  device int32 [n_streams]: handle index per stream.
 *   d_out, cap          device output, grouped by stream in stream order,
 *                       each group in ascending (start, end, label) order;
 *                       positions are relative to the stream's first byte.
 *   d_match_off         device int64 [n_streams + 1]: group offsets.
 *   n_matches           host pointer, receives the grand total.
 * PFSM_EOVERFLOW: *n_matches is the exact total; d_out is unspecified.
 * Device buffers of the batch are kept per stream and grown when a batch
 * needs more.  Synchronises `hip_stream`.
 * Errors: PFSM_EINVAL (arguments, an automaton index outside
 * [0, n_automata), decreasing offsets, a stream longer than 2^31 - 16
 * bytes, n_automata outside [1, 64]), PFSM_EOVERFLOW, PFSM_ENOMEM,
 * PFSM_EHIP.                                                              */
int pfsm_scan_batch(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data,
                    const int64_t *d_stream_off, const int32_t *d_stream_automaton,
                    int32_t n_streams, pfsm_match_t *d_out, int64_t cap, int64_t *d_match_off,
                    int64_t *n_matches, void *hip_stream);

/* pfsm_scan_batch (Section III.A per stream) without any host round trip:
 * every step (planning, one
 * scan launch per automaton, offsets, gather) is enqueued on `hip_stream`
 * and nothing is allocated, so the call can be captured into a HIP graph
 * and replayed.  The grand total is d_match_off[n_streams]; the caller
 * compares it with cap once the stream has reached it.  The device buffers
 * must already be large enough: run pfsm_scan_batch once on the same stream
 * with the same or larger sizes first (PFSM_ENOMEM otherwise).  A captured
 * graph sees later pattern edits of its handles while their
 * PFSM_OPT_LAYOUT_EPOCH is unchanged (pfsm_add_pattern).  A batch
 * whose automaton indices or offsets are invalid reports 0 matches.
 * Errors: PFSM_EINVAL, PFSM_ENOMEM, PFSM_EHIP.                            */
int pfsm_scan_batch_async(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data,
                          const int64_t *d_stream_off, const int32_t *d_stream_automaton,
                          int32_t n_streams, pfsm_match_t *d_out, int64_t cap, int64_t *d_match_off,
                          void *hip_stream);

/* ---------------------------------------------------------------------
 * Launch settings and the autotuner.  Settings change where and how the
 * work runs, never the matches.  A handle's settings apply to its single
 * scans, streams and batches; set them while no scan of the handle is in
 * flight on another thread.
 * --------------------------------------------------------------------- */
enum {
    PFSM_OPT_SEGMENT = 1,             /* bytes of input per segment: 0 = automatic (the input spread
                                         over the resident workgroups, at most 64 KiB), otherwise a
                                         multiple of 16 in [256, 65536]                            */
    PFSM_OPT_WORKGROUPS_PER_CU = 2,   /* resident workgroups per compute unit: 0 = as many as fit   */
    PFSM_OPT_TABLE_BUDGET = 3,        /* DFA: largest transition table kept in LDS, bytes; -1 =
                                         default (96 KiB), 0 = always read the table through L2
                                         (rows of q0's successors still cached in LDS)             */
    PFSM_OPT_PAIR_CACHE = 4,          /* NFA: 1 = cache the sets after two symbols per byte pair
                                         when they fit (default), 0 = never                        */
    PFSM_OPT_MAX_WORKGROUPS_PER_CU = 5, /* read only: how many workgroups fit per compute unit      */
    PFSM_OPT_RESIDENT_TABLE = 6,      /* read only, DFA: 1 when the table is resident in LDS        */
    PFSM_OPT_MERGED_WALKS = 7,        /* DFA with at most 63 states: 1 = tag-merged stepping (one
                                         lookup per distinct active state, Section III.B) for single
                                         scans; 0 = one walk per start (default).  Batches and
                                         streams always walk per start.                            */
    PFSM_OPT_MERGED_COUNT_LIMIT = 8,  /* tag-merged stepping keeps per-start match counts and
                                         output offsets in 32 bits up to this value, and larger
                                         ones in 64 bits in memory: 0 = 2^31 - 1 (default); a small
                                         value exercises the memory paths (results are the same)  */
    PFSM_OPT_LAYOUT_EPOCH = 9         /* read only: advances whenever an edit or a setting moves the
                                         handle's device tables to new buffers or changes a value
                                         its launches carry (the NFA pair cache turned on or off,
                                         a DFA table budget); captured HIP graphs see later edits
                                         only while it stays the same                              */
};

/* Set a writable option (table budget and pair cache rebuild the device
 * caches and synchronise the device).  Errors: PFSM_EINVAL (unknown option
 * or value out of range), PFSM_ENOSYS (option of the other automaton kind),
 * PFSM_ENOMEM, PFSM_EHIP.                                                 */
int pfsm_set_option(pfsm_t *h, int32_t option, int64_t value, void *hip_stream);
/* Read an option.  Errors: PFSM_EINVAL, PFSM_ENOSYS.                      */
int pfsm_get_option(const pfsm_t *h, int32_t option, int64_t *value);

/* What pfsm_tune kept: the settings (-1 for the cache option of the other
 * kind; merged_walks is 0 for NFAs), the time per scan of the sample before
 * and after, the number of settings timed and the sample's match count.   */
typedef struct {
    int64_t segment, workgroups_per_cu, table_budget, pair_cache;
    double ms_before, ms_after;
    int32_t configs, pad;
    int64_t matches;
    int64_t merged_walks;
} pfsm_tune_report;

/* Autotune h on a sample of n device bytes: starting from the current
 * settings, try tag-merged stepping (DFAs that allow it), the cache option
 * (table budget or pair cache), then the workgroups per compute unit, then
 * the segment size, each timed over
 * `reps` scans, and keep each change that saves at least 2 %.  Every
 * setting must reproduce the sample's match list of the starting settings,
 * entry by entry, else PFSM_EINVAL (the settings are then unspecified).
 * Allocates its own output buffer and a host copy of the list;
 * synchronises `hip_stream`.  Errors: PFSM_EINVAL, PFSM_ENOMEM, PFSM_EHIP. */
int pfsm_tune(pfsm_t *h, const uint8_t *d_sample, int64_t n, int32_t reps, pfsm_tune_report *report,
              void *hip_stream);

/* ---------------------------------------------------------------------
 * Streaming scans: chained data partitioning (Section III.D.2).  A stream's
 * bytes are fed in pieces; every instance still live when a piece ends is
 * carried into the next one as its start and state set, so the matches of
 * all pieces together are exactly those of one pfsm_scan of the
 * concatenated bytes, and no piece re-reads earlier bytes.
 * --------------------------------------------------------------------- */
typedef struct pfsm_stream pfsm_stream_t;

/* Open a stream over handle h (which must outlive it) on the current
 * device.  Editing h afterwards (pfsm_add_pattern, pfsm_remove_pattern)
 * makes later pieces fail with PFSM_EINVAL.  Errors: PFSM_EINVAL,
 * PFSM_ENOMEM, PFSM_EHIP.                                                 */
int pfsm_stream_open(pfsm_stream_t **out, pfsm_t *h);

/* Feed the next n bytes (device memory, any alignment) and report the
 * matches that END inside them, in ascending (start, end, label) order,
 * with positions counted from the stream's first byte (starts may lie in
 * earlier pieces).  The stream's total length must stay below 2^31 - 16.
 * n == 0 reports nothing and changes nothing.  PFSM_EOVERFLOW: *n_matches
 * is the exact count, d_out is unspecified, and the stream is left as it
 * was, so the same piece can be fed again with a larger buffer.
 * Synchronises `hip_stream`.  A stream is not safe for concurrent use.
 * Errors: PFSM_EINVAL, PFSM_EOVERFLOW, PFSM_ENOMEM, PFSM_EHIP.            */
int pfsm_stream_feed(pfsm_stream_t *st, const uint8_t *d_piece, int64_t n, pfsm_match_t *d_out,
                     int64_t cap, int64_t *n_matches, void *hip_stream);

/* Bytes fed so far (*position) and the number of live instances carried
 * into the next piece (*n_carried; synchronises `hip_stream`).  Either
 * pointer may be NULL.  Errors: PFSM_EINVAL, PFSM_EHIP.                   */
int pfsm_stream_info(pfsm_stream_t *st, int64_t *position, int64_t *n_carried, void *hip_stream);

/* Free the stream (after the device has finished with it).                */
void pfsm_stream_close(pfsm_stream_t *st);

/* ---------------------------------------------------------------------
 * Serving loop: continuous batching of scan requests (the online use of
 * Section I) against resident handles.  A worker thread admits queued
 * requests, first come first served, into one of two batches while their
 * bytes plus reserved output rows fit `mem_budget` bytes.  The reservation
 * is 1.5 times the matches per byte seen so far on the request's automaton
 * (n/16 before any), plus 256, charged twice for the device and host copies;
 * a request whose matches outgrow it is run again with its exact count.
 * Each batch runs as pfsm_scan_batch does, on a stream of its own; a request
 * arriving while batches run joins the next one as soon as a batch slot and
 * memory free up.  A request larger than the budget runs alone.  Each
 * request's matches are exactly those of pfsm_scan on its bytes alone.
 * --------------------------------------------------------------------- */
typedef struct pfsm_server pfsm_server_t;

/* Counters: batches run, reruns (batches that left requests for a later
 * one), requests finished, their bytes and matches, the largest memory
 * charge in flight, and the worker's time (ns) packing inputs, enqueueing
 * batches and delivering results.                                         */
typedef struct {
    int64_t batches, reruns, requests, bytes, matches, peak_inflight;
    int64_t pack_ns, launch_ns, deliver_ns;
} pfsm_server_stats;

/* Start a server over n_automata handles (1..64), which must outlive it and
 * must not be edited while it runs.  The device is the current one.
 * Errors: PFSM_EINVAL, PFSM_ENOMEM, PFSM_EHIP.                            */
int pfsm_server_create(pfsm_server_t **out, pfsm_t *const *hs, int32_t n_automata, int64_t mem_budget,
                       int32_t max_batch);
/* Queue a scan of n host bytes (copied during the call) against handle
 * `automaton`; *id names the request.  Errors: PFSM_EINVAL.               */
int pfsm_server_submit(pfsm_server_t *sv, int32_t automaton, const uint8_t *bytes, int64_t n, int64_t *id);
/* pfsm_server_submit without the copy: the server reads `bytes` until the
 * request is finished, and the caller keeps them unchanged until then.    */
int pfsm_server_submit_borrowed(pfsm_server_t *sv, int32_t automaton, const uint8_t *bytes, int64_t n,
                                int64_t *id);
/* Block until request `id` is done; *matches (pinned host memory owned by
 * the server, shared with the other requests of its batch and valid until
 * pfsm_server_release; NULL when *n_matches is 0) holds its *n_matches
 * matches in ascending (start, end, label) order.  Errors: PFSM_ENOENT, or
 * the error the request's batch met (PFSM_ENOMEM or PFSM_EHIP when its
 * host output buffer could not be allocated).                              */
int pfsm_server_wait(pfsm_server_t *sv, int64_t id, const pfsm_match_t **matches, int64_t *n_matches);
/* When request `id` was submitted and finished (results on the host), in
 * CLOCK_MONOTONIC nanoseconds; *t_done_ns is 0 while it is not finished.
 * Errors: PFSM_ENOENT.                                                    */
int pfsm_server_times(pfsm_server_t *sv, int64_t id, int64_t *t_submit_ns, int64_t *t_done_ns);
/* Forget a finished request and its matches.  Errors: PFSM_ENOENT,
 * PFSM_EINVAL (not finished).                                             */
int pfsm_server_release(pfsm_server_t *sv, int64_t id);
/* Counters since creation.                                                */
int pfsm_server_stats_get(pfsm_server_t *sv, pfsm_server_stats *out);
/* Finish every queued request, stop the worker and free the server.       */
void pfsm_server_destroy(pfsm_server_t *sv);

/* Work counters of the most recent completed scan of `h` on `hip_stream`
 * (the step counts Section III.C bounds).  Counters are kept per stream,
 * because one handle may scan on several streams at once; the call takes the
 * stream and synchronises it.  No elapsed time is kept: timing every scan
 * would add events to every launch, so callers time with their own events.
 * Errors: PFSM_EINVAL, PFSM_ENOENT (no scan yet), PFSM_EHIP.              */
int pfsm_last_stats(pfsm_t *h, pfsm_stats *out, void *hip_stream);

/* Release a handle and every device buffer it owns.  Waits for the device
 * work that uses them.  NULL is ignored.                                   */
void pfsm_free(pfsm_t *h);

/* Release the buffers the library keeps across calls for batched scans
 * (per device and stream: planning arrays, the match stage, a pinned
 * read-back word).  Waits for the device first.  Call it at teardown, after
 * every batch has finished and before the HIP runtime shuts down; a later
 * batch allocates them again.  Handles, streams and servers are released by
 * their own calls.                                                         */
void pfsm_release_cached(void);

/* Static description of an error code. */
const char *pfsm_strerror(int code);

/* Description of the calling thread's most recent failure ("" if none). */
const char *pfsm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFSM_H */
