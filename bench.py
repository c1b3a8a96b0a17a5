"""Throughput of the all-matches PFSM scan on one MI355X.

A step is one full scan (every start position, every match written in
(start, end, label) order) of one 16 MiB input against a resident 256-state
byte DFA: the random-DFA workload with planted accepting walks.  Inputs are
resident in HBM before timing starts and rotate through 64 distinct copies
(1 GiB), so that the 256 MB Infinity Cache cannot serve them.  The K timed
scans run back to back, replayed from HIP graphs (one scan per input copy),
with events around the timed region; --eager launches them one by one with
events around each instead.

Prints one JSON line with GB/s (value), transitions/s, the single-scan
latency distribution of the synchronous call, the scan kernel's position
against the HBM roofline (and, for the per-start DFA kernel, against the LDS
lookup rate) and the CPU oracle's throughput on the host cores, followed by
the batched, served, long-walk, streamed and autotuned measurements (each
can be skipped).  --workload cfg3 or log measures the NFA union or the
tag-merged log search the same way instead (for profiling runs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# LDS lookups: 32 lane reads (one per bank slot, a wave's 64 addresses in two
# clocks) per clock per CU x 256 CUs x 2.4 GHz, in G lookups/s
LDS_PEAK_GLOOKUPS = 32 * 256 * 2.4
MATCH_BYTES = 12       # one (start, end, label) int32 triple
ROTATE_BYTES = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("cfg2", "cfg3", "log"), default="cfg2",
                    help="cfg2: the 256-state DFA (reported line); cfg3: the 2,000-signature NFA union; "
                         "log: line-bounded log search with tag-merged stepping (profiling runs)")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--latency-iters", type=int, default=10000)
    ap.add_argument("--eager", action="store_true",
                    help="time one launch per scan with events around each, instead of HIP-graph replays")
    ap.add_argument("--overlap-streams", type=int, default=4,
                    help="also time the scans alternating over this many streams (reported as `overlapped`; "
                         "`value` is always one stream); 1 = skip")
    ap.add_argument("--no-cfg3", action="store_true", help="skip the NFA-union (cfg3) measurement")
    ap.add_argument("--cfg3-steps", type=int, default=48)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-replays", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true", help="skip the served (continuous batching) measurement")
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--no-long", action="store_true", help="skip the long-walk (tag-merged vs per-start) measurement")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming (pieces vs whole) measurement")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner report")
    ap.add_argument("--no-small", action="store_true", help="skip the small-scan (cfg1) latency")
    return ap.parse_args()


KERNEL_SOURCES = {
    "cfg2": ["paper_1110_1716_amd/csrc/dfa_scan.hip", "paper_1110_1716_amd/csrc/scan_common.h",
             "paper_1110_1716_amd/csrc/pfsm_dev.h", "paper_1110_1716_amd/csrc/dfa_defer.h"],
    "cfg3": ["paper_1110_1716_amd/csrc/nfa_scan.hip", "paper_1110_1716_amd/csrc/scan_common.h",
             "paper_1110_1716_amd/csrc/pfsm_dev.h", "paper_1110_1716_amd/csrc/dfa_defer.h",
             "paper_1110_1716_amd/csrc/dfa_scan.hip"],
    "log": ["paper_1110_1716_amd/csrc/dfa_merged.hip", "paper_1110_1716_amd/csrc/scan_common.h",
            "paper_1110_1716_amd/csrc/pfsm_dev.h"],
}
TRAFFIC_PROFILE = {"cfg2": "profiles/dfa_scan_cfg2_hbm_traffic.txt",
                   "cfg3": "profiles/nfa_scan_cfg3_hbm_traffic.txt",
                   "log": "profiles/dfa_merged_log_hbm_traffic.txt"}


def measured_traffic(workload: str = "cfg2"):
    """HBM bytes per launch of the scan kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by what it reads
    for a plain copy of known size), or None when the kernel sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE[workload])
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[workload]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    return int(fields["traffic_bytes_per_launch"])


def batched_vs_plain(replays: int):
    """The batched workload: 4,096 streams (64 B-1 MiB, log-uniform) over four
    random byte DFAs (256-4,096 states) and an NFA union of 2,000 signatures.
    Batched = one HIP-graph replay of pfsm_scan_batch_async per batch;
    plain = one synchronous pfsm_scan per stream.  Between the two halves of
    the batched runs the workload's 100 NFA edits are applied (and timed)."""
    import torch
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.cfg4()
    hs = [P.pfsm_load(a) for a in wl.automata]
    d = torch.from_numpy(wl.data).cuda()
    so = torch.from_numpy(wl.stream_off).cuda()
    sa = torch.from_numpy(wl.stream_automaton).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        n0, got, mo = P.pfsm_scan_batch(hs, d, so, sa, stream=s)
        cap = int(n0) * 2 + 4096
        out = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
        mo_g = torch.empty_like(mo)
    s.synchronize()

    def capture():
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            P.pfsm_scan_batch_async(hs, d, so, sa, out, mo_g, stream=s)
        return g

    def graph_runs(g, k):
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):
            e0.record(s)
            for _ in range(k):
                g.replay()
            e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k, int(mo_g[-1].item())

    g = capture()
    ms1, n1 = graph_runs(g, replays)
    if n1 != n0:
        raise SystemExit(f"batched replay count {n1} != {n0}")
    nfa_h = hs[wl.meta["nfa_index"]]
    epoch0 = P.pfsm_get_option(nfa_h, P.PFSM_OPT_LAYOUT_EPOCH)
    lat = []
    for op in wl.ops:
        t0 = time.perf_counter()
        if op[0] == "add":
            P.pfsm_add_pattern(nfa_h, op[1])
        else:
            P.pfsm_remove_pattern(nfa_h, op[1])
        lat.append((time.perf_counter() - t0) * 1e3)
    with torch.cuda.stream(s):
        n2, _, _ = P.pfsm_scan_batch(hs, d, so, sa, stream=s)
    # edits that fit the NFA's buffers keep its layout epoch: the graph
    # captured before them replays the edited automaton
    recaptured = P.pfsm_get_option(nfa_h, P.PFSM_OPT_LAYOUT_EPOCH) != epoch0
    if recaptured:
        g = capture()
    ms2, n3 = graph_runs(g, replays)
    if n3 != n2:
        raise SystemExit(f"batched replay count after the edits {n3} != {n2}")
    # plain: one synchronous scan per stream, same bytes, after the edits
    outp = torch.empty((1 << 20, 3), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = 0
    for i in range(len(wl.stream_automaton)):
        lo, hi = int(wl.stream_off[i]), int(wl.stream_off[i + 1])
        tot += P.pfsm_scan(hs[int(wl.stream_automaton[i])], d[lo:hi], out=outp)[0]
    plain_s = time.perf_counter() - t0
    if tot != n2:
        raise SystemExit(f"plain total {tot} != batched {n2}")
    for h in hs:
        h.free()
    ms = (ms1 + ms2) / 2
    gbs = wl.data.size / (ms / 1e3) / 1e9
    plain = wl.data.size / plain_s / 1e9
    return {"workload": wl.name, "n_streams": int(len(wl.stream_automaton)), "bytes": int(wl.data.size),
            "matches_before_edits": int(n0), "matches_after_edits": int(n2),
            "batched_gbs": round(gbs, 2), "batched_ms": round(ms, 3),
            "batched_ms_before_after_edits": [round(ms1, 3), round(ms2, 3)],
            "plain_gbs": round(plain, 3), "plain_ms": round(plain_s * 1e3, 1),
            "speedup": round(gbs / plain, 2), "launch": "one HIP graph replay per batch",
            "edits": {"ops": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "graph_recaptured": bool(recaptured)}}


def served(n_req: int, n_plain: int = 1000):
    """Served scans: 8 resident automata (4 random 16-state DFAs over abcd, 4
    NFA unions of 2,000 signatures), requests log-uniform 256 B-4 MiB.  The
    closed-loop capacity is the throughput with every request queued at once;
    then requests arrive by a Poisson process at 50 % and 90 % of it.  An
    untimed closed pass over other requests comes first (steady state).
    Latency = scheduled arrival -> results on the host (server timestamps).
    The plain path serves the first `n_plain` capacity requests one at a
    time: copy the bytes to the device, synchronous pfsm_scan, copy the
    matches to the host."""
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.cfg5()
    hs = [P.pfsm_load(a) for a in wl.automata]
    rng = W.rng_for(55)
    sv = P.Server(hs, mem_budget=2 << 30, max_batch=512)
    for a, x in wl.requests(rng, 32):
        sv.wait(sv.submit(a, x, borrow=True))

    def closed(reqs):
        t0 = time.monotonic_ns()
        ids = [sv.submit(a, x, borrow=True) for a, x in reqs]
        done = 0
        for i in ids:
            sv.wait(i, release=False)
            done = max(done, sv.times(i)[1])
            sv.release(i)
        return sum(len(x) for _, x in reqs) / ((done - t0) / 1e9)

    def open_loop(reqs, lam):
        gaps = rng.exponential(1.0 / lam, len(reqs))
        t0 = time.monotonic_ns() + 2_000_000
        arr = t0 + np.cumsum(gaps * 1e9).astype(np.int64)
        ids = []
        for (a, x), t in zip(reqs, arr):
            while time.monotonic_ns() < t:
                pass
            ids.append(sv.submit(a, x, borrow=True))
        lat, last = [], 0
        for i, t in zip(ids, arr):
            sv.wait(i, release=False)
            done = sv.times(i)[1]
            sv.release(i)
            lat.append((done - t) / 1e3)
            last = max(last, done)
        lat = np.asarray(lat)
        nbytes = sum(len(x) for _, x in reqs)
        return {"offered_req_per_s": round(lam, 1), "gbs": round(nbytes / ((last - arr[0]) / 1e9) / 1e9, 3),
                "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
                "requests": len(reqs)}

    # One untimed closed pass first: the server's pool of pinned output
    # buffers grows to its working set (pinning a new buffer is slow), so
    # that the capacity below is the steady state's.
    closed(wl.requests(rng, n_req // 2))
    cap_reqs = wl.requests(rng, n_req)
    mean_bytes = float(np.mean([len(x) for _, x in cap_reqs]))
    capacity = closed(cap_reqs)
    res = {"workload": wl.name, "mean_request_bytes": round(mean_bytes), "capacity_gbs": round(capacity / 1e9, 3)}
    for load in (0.5, 0.9):
        res[f"load_{int(load * 100)}"] = open_loop(wl.requests(rng, n_req), load * capacity / mean_bytes)
    res["server"] = sv.stats()
    res["admission"] = "FIFO into one of two batch slots while bytes + output estimate fit a 2 GiB budget"
    sv.close()

    import torch
    plain_reqs = cap_reqs[:n_plain]
    for a, x in plain_reqs[:16]:
        P.pfsm_scan(hs[a], torch.from_numpy(x).cuda())[1].cpu()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, x in plain_reqs:
        P.pfsm_scan(hs[a], torch.from_numpy(x).cuda())[1].cpu()
    plain_s = time.perf_counter() - t0
    plain_gbs = sum(len(x) for _, x in plain_reqs) / plain_s / 1e9
    res["plain"] = {"gbs": round(plain_gbs, 3), "requests": len(plain_reqs),
                    "path": "per request: host-to-device copy, synchronous pfsm_scan, matches copied to the host"}
    res["capacity_vs_plain"] = round(capacity / 1e9 / plain_gbs, 2)
    for h in hs:
        h.free()
    return res


def _time_async(P, h, x, out, cnt, reps):
    import torch
    P.pfsm_scan_async(h, x, out, cnt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.pfsm_scan_async(h, x, out, cnt)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def long_walks(n: int = 16 << 20):
    """Line-bounded log search (every start lives to the end of its line):
    one walk per start against tag-merged stepping, same input and results."""
    import torch
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.log_search(n=n)
    h = P.pfsm_load(wl.automaton)
    x = torch.from_numpy(wl.data).cuda()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    res = {"workload": wl.name, "n_bytes": n, "seed": wl.seed}
    counts = {}
    try:
        for merged, reps, key in ((0, 3, "per_start"), (1, 20, "merged")):
            P.pfsm_set_option(h, P.PFSM_OPT_MERGED_WALKS, merged)
            m, out = P.pfsm_scan(h, x)
            st = P.pfsm_last_stats(h)
            ms = _time_async(P, h, x, out, cnt, reps)
            counts[key] = (m, int(cnt.item()))
            res[key] = {"ms": round(ms, 3), "GB/s": round(n / ms / 1e6, 3),
                        "transitions_per_s": round(st["transitions"] / ms * 1e3, 1)}
            res["transitions_per_scan"] = int(st["transitions"])
            res["matches"] = int(m)
            del out
    finally:
        h.free()
    if len({v for pair in counts.values() for v in pair}) != 1:
        raise SystemExit(f"long-walk counts differ: {counts}")
    res["speedup"] = round(res["per_start"]["ms"] / res["merged"]["ms"], 2)
    return res


def streamed(piece_sizes=(1 << 20, 4 << 20), passes: int = 3):
    """The bench workload fed through pfsm_stream_feed in pieces (instances
    live at a piece's end carried into the next) against one whole scan."""
    import torch
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.cfg2()
    n = wl.data.size
    h = P.pfsm_load(wl.automaton)
    x = torch.from_numpy(wl.data).cuda()
    out = torch.empty((n // 16 + 4096, 3), dtype=torch.int32, device="cuda")
    res = {"workload": wl.name, "n_bytes": n, "passes": passes}
    try:
        whole, _ = P.pfsm_scan(h, x, out=out)
        for k in piece_sizes:
            with P.Stream(h) as st:
                for lo in range(0, n, k):  # warm-up pass (buffers grown)
                    st.feed(x[lo:lo + k], out=out)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                tot = 0
                for _ in range(passes):
                    for lo in range(0, n, k):
                        m, _ = st.feed(x[lo:lo + k], out=out)
                        tot += m
                dt = (time.perf_counter() - t0) / passes
            if tot != passes * whole:
                raise SystemExit(f"streamed matches {tot // passes} differ from one scan's {whole}")
            res[f"pieces_{k >> 20}MiB"] = {"ms_per_pass": round(dt * 1e3, 3), "GB/s": round(n / dt / 1e9, 2),
                                            "us_per_piece": round(dt * 1e6 / ((n + k - 1) // k), 1)}
        res["matches_per_pass"] = int(whole)
    finally:
        h.free()
    return res


def autotune():
    """What the autotuner keeps for the bench workload (a separate handle;
    the timed handle above runs the default settings)."""
    import torch
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.cfg2()
    h = P.pfsm_load(wl.automaton)
    try:
        rep = P.pfsm_tune(h, torch.from_numpy(wl.data).cuda(), reps=20)
    finally:
        h.free()
    return {k: (round(v, 5) if isinstance(v, float) else v) for k, v in rep.items()}


def small_latency(iters: int):
    """Single-scan latency of the 4 KiB random DFA (launch, scan and count
    read-back of the synchronous call), p50/p99 over `iters` scans."""
    import torch
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.cfg1()
    h = P.pfsm_load(wl.automaton)
    try:
        x = torch.from_numpy(wl.data).cuda()
        m, _ = P.pfsm_scan(h, x)
        out = torch.empty((m + 1024, 3), dtype=torch.int32, device="cuda")
        lat = []
        for _ in range(iters):
            t0 = time.perf_counter()
            P.pfsm_scan(h, x, out=out)
            lat.append(time.perf_counter() - t0)
    finally:
        h.free()
    us = np.array(lat) * 1e6
    return {"workload": wl.name, "n_bytes": int(wl.data.size), "matches": int(m), "iters": iters,
            "p50_us": round(float(np.percentile(us, 50)), 2), "p99_us": round(float(np.percentile(us, 99)), 2),
            "call": "pfsm_scan (synchronous)"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, wl, threads: int, seconds: float):
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.scan(wl.automaton, wl.data, threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return reps, el


def cpu_baseline(wl, seconds: float):
    """The oracle as it is, on the host cores, over repeated passes of the
    same 16 MiB input until `seconds` of wall time have been spent; then on
    one thread for a quarter of that time."""
    import oracle
    threads = oracle.default_threads()
    oracle.scan(wl.automaton, wl.data[:1 << 16], threads=threads)  # load the library
    reps, el = _oracle_rate(oracle, wl, threads, seconds)
    reps1, el1 = _oracle_rate(oracle, wl, 1, seconds / 4)
    return {"value": round(reps * wl.data.size / el / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} full passes over the 16 MiB input ({reps * wl.data.size} bytes, "
                      f"{el:.1f} s wall)",
            "single_thread": {"value": round(reps1 * wl.data.size / el1 / 1e9, 4), "unit": "GB/s",
                              "sample": f"{reps1} full passes, {el1:.1f} s wall"},
            "cpu_model": _cpu_model()}


def time_scans(P, h, xs, out, steps: int, nstreams: int, n_ref: int, ref_rows):
    """K back-to-back scans replayed from HIP graphs: one graph of a scan per
    resident input copy, replayed K // copies times, and one of the remaining
    K % copies scans; events around the whole region on the replaying
    stream.  With nstreams > 1 the scans alternate over that many streams
    (forked and joined inside the graph), so that independent scans overlap.
    Every replayed count and each stream's last match list are checked
    against the eager scan.  Returns (total ms, wall s)."""
    import torch
    dev = out.device
    n_copies = len(xs)
    ns = max(1, nstreams)
    gss = [torch.cuda.Stream() for _ in range(ns)]
    outs = [out] + [torch.empty_like(out) for _ in range(ns - 1)]
    gs = gss[0]
    warm = torch.zeros(2, dtype=torch.int64, device=dev)
    for qi, q in enumerate(gss):
        q.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(q):
            for i in range(2):
                P.pfsm_scan_async(h, xs[i % n_copies], outs[qi], warm[i:i + 1], stream=q)
        q.synchronize()
    cnt_g = torch.zeros(n_copies, dtype=torch.int64, device=dev)
    reps, rest = divmod(steps, n_copies)
    graphs = []
    for m in ([n_copies] if reps else []) + ([rest] if rest else []):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=gs):
            for q in gss[1:]:
                q.wait_stream(gs)  # fork
            for k in range(m):
                P.pfsm_scan_async(h, xs[k], outs[k % ns], cnt_g[k:k + 1], stream=gss[k % ns])
            for q in gss[1:]:
                gs.wait_stream(q)  # join
        graphs.append((g, m))
    with torch.cuda.stream(gs):
        for g, _ in graphs:
            g.replay()  # untimed
    gs.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    with torch.cuda.stream(gs):
        t0.record(gs)
        for _ in range(reps):
            graphs[0][0].replay()
        if rest:
            graphs[-1][0].replay()
        t1.record(gs)
    gs.synchronize()
    wall = time.perf_counter() - wall0
    got = cnt_g[:min(steps, n_copies)].cpu().numpy()
    if not np.all(got == n_ref):
        raise SystemExit(f"scan counts differ between steps: {np.unique(got)} vs {n_ref}")
    for o in outs[:min(ns, steps)]:
        if not np.array_equal(o[:n_ref].cpu().numpy(), ref_rows):
            raise SystemExit("a graph-replayed scan's matches differ from the eager scan's")
    return t0.elapsed_time(t1), wall


def nfa_cfg3(steps: int, cpu_seconds: float, no_cpu: bool):
    """The 2,000-signature NFA union on 64 MiB of Zipf bytes: one-stream
    graph-replayed scans (inputs rotated over 1 GiB of copies), the kernel's
    work counters, the HBM and LDS-lookup rooflines of nfa_scan_kernel, and
    the oracle timed on the host cores over whole passes (whose work counters
    the kernel's must equal)."""
    import torch
    import workloads as W
    import paper_1110_1716_amd as P
    wl = W.cfg3()
    n = wl.data.size
    h = P.pfsm_load(wl.automaton)
    try:
        dev = torch.device("cuda:0")
        host = torch.from_numpy(wl.data.copy())
        xs = [host.to(dev) for _ in range(max(1, ROTATE_BYTES // n))]
        out = torch.empty((n // 64 + 4096, 3), dtype=torch.int32, device=dev)
        n_ref, rows = P.pfsm_scan(h, xs[0], out=out)
        rows = rows.cpu().numpy().copy()
        st = P.pfsm_last_stats(h)
        total_ms, wall = time_scans(P, h, xs, out, steps, 1, n_ref, rows)
        us = total_ms / steps * 1e3
        alg_bytes = n + MATCH_BYTES * n_ref
        res = {"workload": wl.name, "n_bytes": n, "seed": wl.seed, "n_states": int(wl.automaton.n_states),
               "matches_per_scan": int(n_ref), "steps": steps, "us_per_scan": round(us, 3),
               "GB/s": round(n / us / 1e3, 3),
               "transitions_per_scan": int(st["transitions"]), "activations_per_scan": int(st["activations"]),
               "transitions_per_s": round(st["transitions"] / us * 1e6, 1),
               "activations_per_s": round(st["activations"] / us * 1e6, 1),
               "roofline": {"bound": "hbm", "achieved": round(alg_bytes / us / 1e3, 2), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(alg_bytes / us / 1e3 / HBM_PEAK_GBS, 5),
                            "traffic": measured_traffic("cfg3"), "kernel": "nfa_scan_kernel",
                            "launches_per_scan": "nfa_scan_kernel + dfa_place_fused_kernel",
                            "kernel_avg_us": round(us, 3), "alg_bytes_per_launch": int(alg_bytes)},
               "lds_roofline": {"bound": "lds", "achieved": round(st["activations"] / us / 1e3, 2),
                                "peak": LDS_PEAK_GLOOKUPS, "unit": "Glookup/s",
                                "frac": round(st["activations"] / us / 1e3 / LDS_PEAK_GLOOKUPS, 5),
                                "lookups_per_launch": int(st["activations"]),
                                "note": "one state-record lookup per state activation (X)"},
               "wall_s_timed": round(wall, 4)}
        del xs
    finally:
        h.free()
    if not no_cpu:
        import oracle
        threads = oracle.default_threads()
        reps, t0, wk = 0, time.perf_counter(), None
        while True:
            ref, wk = oracle.scan(wl.automaton, wl.data, threads=threads)
            reps += 1
            el = time.perf_counter() - t0
            if el >= cpu_seconds:
                break
        if len(ref) != n_ref or wk["T"] != res["transitions_per_scan"] or wk["X"] != res["activations_per_scan"]:
            raise SystemExit(f"cfg3: GPU {n_ref} matches / {res['transitions_per_scan']} T / "
                             f"{res['activations_per_scan']} X, oracle {len(ref)} / {wk['T']} / {wk['X']}")
        res["cpu_baseline"] = {"value": round(reps * n / el / 1e9, 5), "unit": "GB/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{reps} full passes over the 64 MiB input ({reps * n} bytes, {el:.1f} s wall); "
                                         "its matches, T and X equal the GPU scan's",
                               "activations_per_s": round(wk["X"] * reps / el, 1), "cpu_model": _cpu_model()}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the scan shards by input segment; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    import paper_1110_1716_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = {"cfg2": W.cfg2, "cfg3": W.cfg3, "log": W.log_search}[args.workload]()
    n = wl.data.size
    h = P.pfsm_load(wl.automaton)
    kernel = {"cfg2": "dfa_scan_kernel", "cfg3": "nfa_scan_kernel", "log": "dfa_merged_kernel"}[args.workload]
    # the launches of one scan, timed together as kernel_avg_us
    launches = {"cfg2": "dfa_scan_kernel + dfa_place_fused_kernel", "cfg3": "nfa_scan_kernel + dfa_place_fused_kernel",
                "log": "dfa_merged_kernel (count) + merged_seg_scan_kernel + dfa_merged_kernel (write)"}[args.workload]
    if args.workload == "log":
        P.pfsm_set_option(h, P.PFSM_OPT_MERGED_WALKS, 1)

    host = torch.from_numpy(wl.data.copy())
    n_copies = max(1, ROTATE_BYTES // n)
    xs = [host.to(dev) for _ in range(n_copies)]
    cap = n // 8 + 4096 if args.workload != "log" else n + 4096
    out = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    counts = torch.zeros(args.steps + args.warmup, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    if args.calib_copy_mib:
        a_ = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()
        del a_, b_

    # reference result and work counters of one scan (from the kernel's own counters)
    n_ref, ref_rows = P.pfsm_scan(h, xs[0], out=out)
    ref_rows = ref_rows.cpu().numpy().copy()
    stats = P.pfsm_last_stats(h)
    transitions = stats["transitions"]

    for i in range(args.warmup):
        P.pfsm_scan_async(h, xs[i % n_copies], out, counts[i:i + 1])
    torch.cuda.synchronize()

    overlapped = None
    if args.eager:
        # one launch per scan, events around each
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t_start.record(stream)
        for i in range(args.steps):
            k = args.warmup + i
            ev[i][0].record(stream)
            P.pfsm_scan_async(h, xs[k % n_copies], out, counts[k:k + 1])
            ev[i][1].record(stream)
        t_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        total_ms = t_start.elapsed_time(t_end)
        kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
        got = counts.cpu().numpy()
        if not np.all(got == n_ref):
            raise SystemExit(f"scan counts differ between steps: {np.unique(got)} vs {n_ref}")
        timing = "one launch per scan; events around each launch"
    else:
        # `value`: the scans back to back on one stream, replayed from HIP
        # graphs; the overlapped rate (independent scans alternating over
        # several streams) is reported beside it
        total_ms, wall = time_scans(P, h, xs, out, args.steps, 1, n_ref, ref_rows)
        kern_ms = np.array([total_ms / args.steps])
        timing = "HIP-graph replays of back-to-back scans on one stream; events around the timed region"
        if args.overlap_streams > 1:
            o_ms, _ = time_scans(P, h, xs, out, args.steps, args.overlap_streams, n_ref, ref_rows)
            overlapped = {"streams": args.overlap_streams, "GB/s": round(n * args.steps / (o_ms / 1e3) / 1e9, 2),
                          "us_per_scan": round(o_ms / args.steps * 1e3, 3),
                          "note": "independent scans alternating over several streams inside the graph, so that "
                                  "one scan's workgroups fill the compute units the previous one leaves idle"}

    ms_per_step = total_ms / args.steps
    gbs = n * args.steps / (total_ms / 1e3) / 1e9
    tps = transitions * args.steps / (total_ms / 1e3)

    # single-scan latency of the synchronous call (launch + count read-back)
    lat = []
    for i in range(args.latency_iters):
        t0 = time.perf_counter()
        P.pfsm_scan(h, xs[i % n_copies], out=out)
        lat.append(time.perf_counter() - t0)
    lat_us = np.array(lat) * 1e6

    kern_avg_s = float(kern_ms.mean()) / 1e3
    alg_bytes = n + MATCH_BYTES * n_ref
    achieved = alg_bytes / kern_avg_s / 1e9

    res = {
        "metric": "input GB/s and transitions/s per MI355X (batched vs plain); p50/p99 scan latency",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_bytes": n, "seed": wl.seed,
                   "n_states": int(wl.automaton.n_states), "kind": wl.automaton.kind,
                   "matches_per_scan": int(n_ref), "resident_input_copies": n_copies,
                   "streams": 1 if not args.eager else "eager"},
        "transitions_per_s": round(tps, 1),
        "transitions_per_scan": int(transitions),
        "latency_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                       "p99": round(float(np.percentile(lat_us, 99)), 2),
                       "iters": args.latency_iters, "call": "pfsm_scan (synchronous)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload),
                     "kernel": kernel, "launches_per_scan": launches, "kernel_avg_us": round(kern_avg_s * 1e6, 3),
                     "alg_bytes_per_launch": int(alg_bytes)},
        "lds_roofline": ({"bound": "lds", "achieved": round(transitions / kern_avg_s / 1e9, 2),
                          "peak": LDS_PEAK_GLOOKUPS, "unit": "Glookup/s",
                          "frac": round(transitions / kern_avg_s / 1e9 / LDS_PEAK_GLOOKUPS, 4),
                          "lookups_per_launch": int(transitions),
                          "note": "one table lookup per instance-step (T)"}
                         if kernel == "dfa_scan_kernel" else
                         {"bound": "lds", "achieved": round(stats["activations"] / kern_avg_s / 1e9, 2),
                          "peak": LDS_PEAK_GLOOKUPS, "unit": "Glookup/s",
                          "frac": round(stats["activations"] / kern_avg_s / 1e9 / LDS_PEAK_GLOOKUPS, 5),
                          "lookups_per_launch": int(stats["activations"]),
                          "note": "one state-record lookup per state activation (X)"}
                         if kernel == "nfa_scan_kernel" else None),
        "wall_s_timed": round(wall, 4),
        "timing": timing,
        "overlapped": overlapped,
    }
    h.free()
    del xs
    torch.cuda.empty_cache()
    sections = [("cfg3", args.no_cfg3 or args.workload != "cfg2",
                 lambda: nfa_cfg3(args.cfg3_steps, args.cpu_seconds, args.no_cpu)),
                ("batched", args.no_batch, lambda: batched_vs_plain(args.batch_replays)),
                ("served", args.no_serve, lambda: served(args.serve_requests)),
                ("long_walks", args.no_long, long_walks),
                ("streamed", args.no_stream, streamed),
                ("autotune", args.no_tune, autotune),
                ("latency_cfg1", args.no_small, lambda: small_latency(10000)),
                ("cpu_baseline", args.no_cpu, lambda: cpu_baseline(wl, args.cpu_seconds))]
    print(f"bench: {args.workload} scan timed", file=sys.stderr, flush=True)
    for key, skip, fn in sections:
        if not skip:
            res[key] = fn()
            print(f"bench: {key} done", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
