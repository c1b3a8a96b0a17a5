"""GPU parity of the batched scan (pfsm_scan_batch) against the CPU oracle,
stream by stream (bit-exact match lists, grouped by stream)."""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.regex import regex_nfa

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1110_1716_amd as P
    P.load_library()
    return P


def pack(streams):
    """Concatenate byte streams; offsets int64 [n+1] (streams start at any byte)."""
    off = np.zeros(len(streams) + 1, np.int64)
    for i, s in enumerate(streams):
        off[i + 1] = off[i] + len(s)
    data = np.concatenate([np.frombuffer(bytes(s), np.uint8) if isinstance(s, (bytes, bytearray))
                           else np.asarray(s, np.uint8) for s in streams]) if streams else np.zeros(0, np.uint8)
    return data, off


def run_batch(P, automata, streams, aut_of, out_rows=None):
    data, off = pack(streams)
    hs = [P.pfsm_load(a) for a in automata]
    try:
        d = torch.from_numpy(data.copy() if data.size else np.zeros(16, np.uint8)).cuda()
        so = torch.from_numpy(off).cuda()
        sa = torch.from_numpy(np.asarray(aut_of, np.int32)).cuda()
        out = None if out_rows is None else torch.empty((out_rows, 3), dtype=torch.int32, device="cuda")
        n, got, mo = P.pfsm_scan_batch(hs, d, so, sa, out=out)
        return n, got.cpu().numpy(), mo.cpu().numpy()
    finally:
        for h in hs:
            h.free()


def check_batch(P, automata, streams, aut_of):
    n, got, mo = run_batch(P, automata, streams, aut_of)
    assert mo[0] == 0 and mo[-1] == n == len(got)
    for i, s in enumerate(streams):
        ref, _ = oracle.scan(automata[aut_of[i]], np.frombuffer(bytes(s), np.uint8) if isinstance(s, bytes) else s)
        grp = got[mo[i]:mo[i + 1]]
        assert grp.shape == ref.shape, (i, len(s), grp.shape, ref.shape)
        assert np.array_equal(grp, ref), i
    return n


def mixed_automata():
    return [W.cfg1(seed=11).automaton, W.cfg2(seed=12, n=1 << 16).automaton,
            W.cfg3(seed=13, n=1 << 16, n_patterns=150).automaton,
            regex_nfa([(b"a*c", 0), (b"ac", 1), (b"a(ca)*b", 2)])]


def stream_for(rng, aut_idx, n):
    if aut_idx in (0, 3):
        return bytes(rng.choice(list(b"abcd"), n).astype(np.uint8))
    return rng.integers(0, 256, n, dtype=np.uint8).tobytes()


def test_mixed_small(P):
    rng = np.random.default_rng(1)
    autos = mixed_automata()
    lens = [0, 1, 2, 3, 15, 16, 17, 100, 1000, 4095, 5000, 0, 7, 33333]
    aut_of = [int(rng.integers(0, len(autos))) for _ in lens]
    streams = [stream_for(rng, a, n) for a, n in zip(aut_of, lens)]
    check_batch(P, autos, streams, aut_of)


def test_streams_longer_than_a_segment(P):
    rng = np.random.default_rng(2)
    wl = W.cfg2(seed=21, n=600_000)
    nfa = W.cfg3(seed=22, n=1 << 16, n_patterns=200).automaton
    streams = [wl.data[:200_000].tobytes(), wl.data[200_001:500_000].tobytes(),
               rng.integers(0, 256, 150_007, dtype=np.uint8).tobytes(), wl.data[3:70_000].tobytes()]
    check_batch(P, [wl.automaton, nfa], streams, [0, 0, 1, 1])


def test_many_small_streams(P):
    rng = np.random.default_rng(3)
    autos = mixed_automata()
    n = 700
    aut_of = [int(a) for a in rng.integers(0, len(autos), n)]
    lens = np.exp(rng.uniform(np.log(1), np.log(3000), n)).astype(int)
    streams = [stream_for(rng, a, int(k)) for a, k in zip(aut_of, lens)]
    check_batch(P, autos, streams, aut_of)


def test_batch_equals_plain_scans(P):
    rng = np.random.default_rng(4)
    wl = W.cfg2(seed=41, n=1 << 18)
    h = P.pfsm_load(wl.automaton)
    cuts = np.sort(rng.integers(0, wl.data.size, 9))
    streams = [wl.data[a:b].tobytes() for a, b in zip(np.r_[0, cuts], np.r_[cuts, wl.data.size])]
    n, got, mo = run_batch(P, [wl.automaton], streams, [0] * len(streams))
    for i, s in enumerate(streams):
        x = torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() if s else torch.zeros(0, dtype=torch.uint8,
                                                                                              device="cuda")
        if len(s) == 0:
            assert mo[i + 1] == mo[i]
            continue
        k, plain = P.pfsm_scan(h, x)
        assert np.array_equal(got[mo[i]:mo[i + 1]], plain.cpu().numpy()), i
    h.free()


def test_overflow_reports_exact_count(P):
    rng = np.random.default_rng(5)
    autos = [W.cfg2(seed=51, n=1 << 16).automaton]
    streams = [rng.integers(0, 256, 50_000, dtype=np.uint8).tobytes() for _ in range(3)]
    total = sum(len(oracle.scan(autos[0], np.frombuffer(s, np.uint8))[0]) for s in streams)
    assert total > 10
    with pytest.raises(P.PfsmError) as ei:
        run_batch(P, autos, streams, [0, 0, 0], out_rows=10)
    assert ei.value.code == P.PFSM_EOVERFLOW
    n, got, mo = run_batch(P, autos, streams, [0, 0, 0], out_rows=total)
    assert n == total


def test_bad_automaton_index(P):
    autos = [W.cfg1(seed=11).automaton]
    with pytest.raises(P.PfsmError) as ei:
        run_batch(P, autos, [b"abcd", b"abca"], [0, 1])
    assert ei.value.code == P.PFSM_EINVAL


def test_empty_batch(P):
    autos = [W.cfg1(seed=11).automaton]
    n, got, mo = run_batch(P, autos, [], [])
    assert n == 0 and list(mo) == [0]


def test_repeated_batches_same_buffers(P):
    """Back-to-back batches reuse the device workspaces (epochs, tickets)."""
    rng = np.random.default_rng(6)
    autos = mixed_automata()
    for rep in range(3):
        n = 40 + 30 * rep
        aut_of = [int(a) for a in rng.integers(0, len(autos), n)]
        streams = [stream_for(rng, a, int(rng.integers(0, 9000))) for a in aut_of]
        check_batch(P, autos, streams, aut_of)


def _cfg4_refs(wl, removed, added):
    """Oracle lists per stream for cfg4 after NFA edits: the union of the
    base NFA and every added pattern, without the removed labels."""
    from oracle import compose
    nfa_i = wl.meta["nfa_index"]
    nfa = compose.union([wl.automata[nfa_i]] + added) if added else wl.automata[nfa_i]
    refs = []
    for s in range(len(wl.stream_automaton)):
        x = wl.data[wl.stream_off[s]:wl.stream_off[s + 1]]
        a = int(wl.stream_automaton[s])
        ref, _ = oracle.scan(nfa if a == nfa_i else wl.automata[a], x)
        if a == nfa_i:
            for lab in removed:
                ref = compose.drop_label(ref, lab)
        refs.append(ref)
    return refs


def _batch_lists(P, hs, wl):
    d = torch.from_numpy(wl.data.copy()).cuda()
    so = torch.from_numpy(wl.stream_off).cuda()
    sa = torch.from_numpy(wl.stream_automaton).cuda()
    n, got, mo = P.pfsm_scan_batch(hs, d, so, sa)
    got, mo = got.cpu().numpy(), mo.cpu().numpy()
    return [got[mo[s]:mo[s + 1]] for s in range(len(wl.stream_automaton))]


def test_cfg4_small_with_edits(P):
    """The batched workload (four DFAs of 256-4,096 states and an NFA union)
    at a small size, before and after add/remove edits of the NFA."""
    wl = W.cfg4(seed=44, n_streams=80, len_hi=1 << 15, n_patterns=150, n_ops=8)
    hs = [P.pfsm_load(a) for a in wl.automata]
    try:
        refs = _cfg4_refs(wl, [], [])
        for s, grp in enumerate(_batch_lists(P, hs, wl)):
            assert np.array_equal(grp, refs[s]), s
        nfa_h = hs[wl.meta["nfa_index"]]
        removed, added = [], []
        for op in wl.ops:
            if op[0] == "add":
                P.pfsm_add_pattern(nfa_h, op[1])
                added.append(op[1])
            else:
                P.pfsm_remove_pattern(nfa_h, op[1])
                removed.append(op[1])
        refs = _cfg4_refs(wl, removed, added)
        for s, grp in enumerate(_batch_lists(P, hs, wl)):
            assert np.array_equal(grp, refs[s]), s
    finally:
        for h in hs:
            h.free()


def test_graph_capture_replays(P):
    """pfsm_scan_batch_async captured in a HIP graph: every replay, with eager
    scans in between, equals the eager batch."""
    wl = W.cfg4(seed=45, n_streams=60, len_hi=1 << 15, n_patterns=100, n_ops=0)
    hs = [P.pfsm_load(a) for a in wl.automata]
    try:
        s = torch.cuda.Stream()
        d = torch.from_numpy(wl.data.copy()).cuda()
        so = torch.from_numpy(wl.stream_off).cuda()
        sa = torch.from_numpy(wl.stream_automaton).cuda()
        cap = wl.data.size // 16 + 1024
        with torch.cuda.stream(s):
            out_e = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
            n_e, got_e, mo_e = P.pfsm_scan_batch(hs, d, so, sa, out=out_e, stream=s)
            got_e, mo_e = got_e.cpu().numpy().copy(), mo_e.cpu().numpy().copy()
            out_g = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
            mo_g = torch.empty(len(wl.stream_automaton) + 1, dtype=torch.int64, device="cuda")
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            P.pfsm_scan_batch_async(hs, d, so, sa, out_g, mo_g, stream=s)
        other = W.cfg2(seed=46, n=1 << 17)
        h2 = P.pfsm_load(other.automaton)
        x2 = torch.from_numpy(other.data.copy()).cuda()
        for rep in range(3):
            out_g.fill_(-1)
            mo_g.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(mo_g.cpu().numpy(), mo_e), rep
            assert np.array_equal(out_g[:n_e].cpu().numpy(), got_e), rep
            P.pfsm_scan(h2, x2)  # eager work between replays
            P.pfsm_scan_batch(hs, d, so, sa, stream=s)
            torch.cuda.synchronize()
        h2.free()
    finally:
        for h in hs:
            h.free()


def test_cfg4_full_size_with_edits(P):
    """The batched workload at its stated size: 4,096 streams of 64 B-1 MiB
    (about 460 MB) over four DFAs of 256-4,096 states and a 2,000-signature
    NFA union; every stream's list equals the oracle's before and after the
    workload's 100 add/remove edits of the NFA."""
    wl = W.cfg4()
    assert len(wl.stream_automaton) == 4096 and len(wl.ops) == 100
    print(f"cfg4 full: {len(wl.stream_automaton)} streams, {wl.data.size} bytes", flush=True)
    hs = [P.pfsm_load(a) for a in wl.automata]
    try:
        got = _batch_lists(P, hs, wl)
        refs = _cfg4_refs(wl, [], [])
        for s in range(len(refs)):
            assert np.array_equal(got[s], refs[s]), s
        nfa_h = hs[wl.meta["nfa_index"]]
        removed, added = [], []
        for op in wl.ops:
            if op[0] == "add":
                P.pfsm_add_pattern(nfa_h, op[1])
                added.append(op[1])
            else:
                P.pfsm_remove_pattern(nfa_h, op[1])
                removed.append(op[1])
        got = _batch_lists(P, hs, wl)
        refs = _cfg4_refs(wl, removed, added)
        for s in range(len(refs)):
            assert np.array_equal(got[s], refs[s]), s
    finally:
        for h in hs:
            h.free()


def test_graph_replay_sees_edits_until_the_layout_moves(P):
    """A batch captured in a HIP graph, then NFA adds/removes and a DFA label
    removal that fit the handles' buffers: the layout epoch stays and every
    replay equals the oracle of the edited automata.  An add that outgrows
    the NFA's buffers advances its epoch: the old graph still replays its
    (unchanged) old buffers, an eager batch sees the new pattern, and a graph
    captured again does too."""
    from oracle import compose
    wl = W.cfg4(seed=47, n_streams=60, len_hi=1 << 15, n_patterns=100, n_ops=8)
    hs = [P.pfsm_load(a) for a in wl.automata]
    nfa_i = wl.meta["nfa_index"]
    nfa_h = hs[nfa_i]
    # a label of the 256-state DFA (table resident in LDS) and of the
    # 4,096-state one (table read through L2)
    dfa_labs = {0: int(np.asarray(wl.automata[0].final_labels)[0]),
                3: int(np.asarray(wl.automata[3].final_labels)[-1])}
    try:
        s = torch.cuda.Stream()
        d = torch.from_numpy(wl.data.copy()).cuda()
        so = torch.from_numpy(wl.stream_off).cuda()
        sa = torch.from_numpy(wl.stream_automaton).cuda()
        cap = wl.data.size // 16 + 1024
        n_s = len(wl.stream_automaton)
        with torch.cuda.stream(s):
            out_g = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
            mo_g = torch.empty(n_s + 1, dtype=torch.int64, device="cuda")
            P.pfsm_scan_batch(hs, d, so, sa, stream=s)
        s.synchronize()

        def capture():
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                P.pfsm_scan_batch_async(hs, d, so, sa, out_g, mo_g, stream=s)
            return g

        def replay_lists(g):
            out_g.fill_(-1)
            mo_g.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got, mo = out_g.cpu().numpy(), mo_g.cpu().numpy()
            return [got[mo[i]:mo[i + 1]] for i in range(n_s)]

        def refs_for(removed, added, dfa_removed):
            refs = _cfg4_refs(wl, removed, added)
            for i in range(n_s):
                a = int(wl.stream_automaton[i])
                if a in dfa_labs and dfa_removed:
                    refs[i] = compose.drop_label(refs[i], dfa_labs[a])
            return refs

        def same(lists, refs):
            for i in range(n_s):
                assert np.array_equal(lists[i], refs[i]), i

        g = capture()
        same(replay_lists(g), refs_for([], [], False))
        e_nfa = P.pfsm_get_option(nfa_h, P.PFSM_OPT_LAYOUT_EPOCH)
        e_dfa = {a: P.pfsm_get_option(hs[a], P.PFSM_OPT_LAYOUT_EPOCH) for a in dfa_labs}
        removed, added = [], []
        for op in wl.ops:
            if op[0] == "add":
                P.pfsm_add_pattern(nfa_h, op[1])
                added.append(op[1])
            else:
                P.pfsm_remove_pattern(nfa_h, op[1])
                removed.append(op[1])
        for a, lab in dfa_labs.items():
            P.pfsm_remove_pattern(hs[a], lab)
        assert P.pfsm_get_option(nfa_h, P.PFSM_OPT_LAYOUT_EPOCH) == e_nfa
        for a in dfa_labs:
            assert P.pfsm_get_option(hs[a], P.PFSM_OPT_LAYOUT_EPOCH) == e_dfa[a]
        edited = refs_for(removed, added, True)
        for rep in range(2):
            same(replay_lists(g), edited)
            P.pfsm_scan_batch(hs, d, so, sa, stream=s)  # eager work between replays
            torch.cuda.synchronize()

        # an add far larger than the union so far: the NFA's buffers move
        big = W.union_nfa(W.signature_union(np.random.default_rng(48), 300, label_base=5000))
        P.pfsm_add_pattern(nfa_h, big)
        assert P.pfsm_get_option(nfa_h, P.PFSM_OPT_LAYOUT_EPOCH) > e_nfa
        same(replay_lists(g), edited)  # the old buffers, as they were
        grown = refs_for(removed, added + [big], True)
        n, got, mo = P.pfsm_scan_batch(hs, d, so, sa, stream=s)
        got, mo = got.cpu().numpy(), mo.cpu().numpy()
        same([got[mo[i]:mo[i + 1]] for i in range(n_s)], grown)
        del g
        g2 = capture()
        same(replay_lists(g2), grown)
    finally:
        for h in hs:
            h.free()
