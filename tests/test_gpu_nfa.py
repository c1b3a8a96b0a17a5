"""GPU parity of the NFA scan against the CPU oracle (bit-exact match lists)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import compose
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


def dev(x):
    a = np.array(np.frombuffer(bytes(x), np.uint8)) if isinstance(x, (bytes, bytearray)) else np.ascontiguousarray(x)
    return torch.from_numpy(a).cuda()


def check(P, fsm, x, work=True):
    ref, wk = oracle.scan(fsm, x)
    h = P.pfsm_load(fsm)
    try:
        n, out = P.pfsm_scan(h, dev(x))
        got = out.cpu().numpy()
        stats = P.pfsm_last_stats(h) if len(x) else None
    finally:
        h.free()
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.array_equal(got, ref)
    if work and stats is not None:
        assert stats["transitions"] == wk["T"]
        assert stats["activations"] == wk["X"]
        assert stats["matches"] == len(ref)
    return ref


def test_fig2_nfa(P):
    ref = check(P, W.fig1_nfa(), W.FIG2_INPUT)
    assert len(ref) == 10


@pytest.mark.parametrize("pat", [b"a*c", b"(ab|a)*b{1,3}", b"[a-c]+d?", b"a.{0,3}b", b"(a|b)*abb",
                                 b"((a|b)(c|d))+", b"(a*)*b", b"(a|b|c|d)*d"])
def test_regex_nfas(P, pat):
    rng = np.random.default_rng(len(pat))
    x = bytes(rng.choice(list(b"abcd"), 3000).astype(np.uint8))
    check(P, regex_nfa([(pat, 3)]), x)


def test_regex_union(P):
    pats = [(b"a*c", 0), (b"ac", 1), (b"a(ca)*b", 2), (b"(a|b)*abb", 7), (b"d{2,}", 9)]
    rng = np.random.default_rng(4)
    x = bytes(rng.choice(list(b"abcd"), 20000).astype(np.uint8))
    check(P, regex_nfa(pats), x)


@pytest.mark.parametrize("seed", range(10))
def test_random_nfas(P, seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(2, 14))
    fsm = W.random_nfa(rng, n, list(b"abc"), n_edges=int(rng.integers(n, 3 * n)), p_eps=0.2,
                       n_finals=int(rng.integers(1, 4)))
    x = bytes(rng.choice(list(b"abcd"), int(rng.integers(1, 6000))).astype(np.uint8))
    check(P, fsm, x)


@pytest.mark.parametrize("n", [1, 2, 3, 4095, 4097, 70001])
def test_ragged_sizes(P, n):
    wl = W.cfg3(seed=31, n=max(n, 64), n_patterns=150, plant_rate=2e-3)
    check(P, wl.automaton, wl.data[:n])


def gap_union(gap_max):
    """Signature chains with one any-byte gap each: chains of one, two and
    three states after the gap's exit edge E, and byte classes on E and on
    the chain's first edge."""
    S = W.Signature
    sigs = [S([[97], [98]], 1, 0),                          # a .{0,g} b
            S([[97], [98], [99]], 1, 1),                    # a .{0,g} b c
            S([[99], [97, 98], [98], [97], [99]], 2, 2),    # c [ab] .{0,g} b a c
            S([[100], [97, 98, 99], [97, 99]], 1, 3)]       # d .{0,g} [abc] [ac]
    return W.union_nfa(sigs, gap_max=gap_max)


@pytest.mark.parametrize("gap_max", [8, 64, 100])
@pytest.mark.parametrize("n", [777, 5000])
def test_gap_chains(P, gap_max, n):
    """Gap walks finished in one pass: many exits per gap, walks cut off by
    the end of the input, gaps longer than one pass covers."""
    rng = np.random.default_rng(gap_max * 7 + n)
    x = bytes(rng.choice(list(b"abcd"), n, p=[0.4, 0.3, 0.2, 0.1]).astype(np.uint8))
    ref = check(P, gap_union(gap_max), x)
    assert len(ref) > 0


def test_cfg3_small(P):
    wl = W.cfg3(seed=33, n=1 << 20, n_patterns=300, plant_rate=5e-4)
    ref = check(P, wl.automaton, wl.data)
    assert len(ref) > 100


def test_cfg3_full(P):
    wl = W.cfg3()
    ref = check(P, wl.automaton, wl.data)
    assert len(ref) >= len(wl.meta["plants"])


def test_unaligned_input(P):
    wl = W.cfg3(seed=34, n=1 << 16, n_patterns=100, plant_rate=2e-3)
    ref, _ = oracle.scan(wl.automaton, wl.data[5:])
    h = P.pfsm_load(wl.automaton)
    n, out = P.pfsm_scan(h, dev(wl.data)[5:])
    h.free()
    assert np.array_equal(out.cpu().numpy(), ref)


def test_dense_matches(P):
    """a+ on a^3000: every substring matches; every segment overflows its buffer."""
    ref = check(P, regex_nfa([(b"a+", 1)]), b"a" * 3000)
    assert len(ref) == 3000 * 3001 // 2


def test_wide_sets_without_pair_cache(P):
    """600 two-symbol patterns under one initial state: sets of 600 states,
    byte-pair cache over budget, every instance replayed by a workgroup."""
    k = 600
    edges = []
    for i in range(k):
        s, t, u = 1 + 3 * i, 2 + 3 * i, 3 + 3 * i
        edges += [(0, -1, s), (s, 0, t), (t, 0, u)]
    src, cls, dst = zip(*edges)
    fsm = W.build_nfa(1 + 3 * k, 0, src, cls, dst, [list(range(256))],
                      {3 + 3 * i: [i] for i in range(k)})
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, 700, dtype=np.uint8)
    ref = check(P, fsm, x)
    assert len(ref) == 699 * k


def test_add_then_remove(P):
    wl = W.cfg3(seed=35, n=1 << 18, n_patterns=200, plant_rate=1e-3)
    base = wl.automaton
    rng = W.rng_for(99)
    extra = W.signature_union(rng, n_patterns=3, label_base=5000)
    pat = W.union_nfa(extra)
    # plant the extra patterns
    x = wl.data.copy()
    for j, sig in enumerate(extra):
        inst = bytes(s[0] for s in sig.edge_sets)
        x[1000 + 4000 * j:1000 + 4000 * j + len(inst)] = np.frombuffer(inst, np.uint8)
    ref_base, _ = oracle.scan(base, x)
    ref_union, _ = oracle.scan(compose.union([base, pat]), x)
    assert len(ref_union) > len(ref_base)
    h = P.pfsm_load(base)
    xd = dev(x)
    assert np.array_equal(P.pfsm_scan(h, xd)[1].cpu().numpy(), ref_base)
    P.pfsm_add_pattern(h, pat)
    assert np.array_equal(P.pfsm_scan(h, xd)[1].cpu().numpy(), ref_union)
    with pytest.raises(P.PfsmError) as ei:
        P.pfsm_add_pattern(h, pat)
    assert ei.value.code == P.PFSM_EEXIST
    P.pfsm_remove_pattern(h, 5001)  # cuts the added pattern (all its labels)
    assert np.array_equal(P.pfsm_scan(h, xd)[1].cpu().numpy(), ref_base)
    # a label of the loaded automaton is disabled
    lab = int(ref_base[0, 2])
    P.pfsm_remove_pattern(h, lab)
    assert np.array_equal(P.pfsm_scan(h, xd)[1].cpu().numpy(), compose.drop_label(ref_base, lab))
    with pytest.raises(P.PfsmError) as ei:
        P.pfsm_remove_pattern(h, lab)
    assert ei.value.code == P.PFSM_ENOENT
    h.free()


def test_dfa_and_its_nfa_form_agree(P):
    wl = W.cfg2(seed=12, n=1 << 20)
    nfa = W.dfa_as_nfa(wl.automaton)
    ref = check(P, nfa, wl.data)
    ref_dfa, _ = oracle.scan(wl.automaton, wl.data)
    assert np.array_equal(ref, ref_dfa)


def test_back_to_back_async(P):
    wl = W.cfg3(seed=36, n=3 << 20, n_patterns=300, plant_rate=5e-4)
    h = P.pfsm_load(wl.automaton)
    sizes = [3 << 20, 777, 1 << 20]
    outs = [torch.empty((s // 16 + 1024, 3), dtype=torch.int32, device="cuda") for s in sizes]
    cnts = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    xs = [dev(wl.data[:s]) for s in sizes]
    for i in range(len(sizes)):
        P.pfsm_scan_async(h, xs[i], outs[i], cnts[i:i + 1])
    torch.cuda.synchronize()
    for i, s in enumerate(sizes):
        ref, _ = oracle.scan(wl.automaton, wl.data[:s])
        c = int(cnts[i].item())
        assert c == len(ref) and np.array_equal(outs[i][:c].cpu().numpy(), ref)
    h.free()


def test_replay_list_overflow_recounted(P):
    # sets larger than a lane keeps at every start: more replays than the
    # list holds, so the segment falls back to fresh per-start walks
    pats = [(b"[a-d]*a", 0), (b"[a-d]*b", 1), (b"[a-d]*c[a-d]", 2), (b"[ab]*dd", 3), (b"(a|c)*b[a-d]", 4),
            (b"[a-d]*ab", 5), (b"[cd]*a", 6)]
    fsm = regex_nfa(pats)
    rng = np.random.default_rng(41)
    x = rng.choice(list(b"abcd"), 16384).astype(np.uint8)
    x[rng.random(x.size) < 0.02] = ord("e")  # walks end at an 'e'
    ref, wk = oracle.scan(fsm, x)
    h = P.pfsm_load(fsm)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, 4096)
        n, out = P.pfsm_scan(h, dev(x))
        assert np.array_equal(out.cpu().numpy(), ref)
        st = P.pfsm_last_stats(h)
        assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref))
    finally:
        h.free()


@pytest.mark.parametrize("pat", [b"a.{0,3}b", b"(ab|cd)+", b"a(b|c)*d"])
def test_replay_list_overflow_mid_segment(P, pat):
    # one full 4 KiB window per segment, four waves listing replays at once:
    # the list overflows before its first run while the matches still fit
    # the buffer, so only the dropped replays can force the recount
    rng = np.random.default_rng(len(pat))
    x = rng.choice(list(b"abcd"), 3000).astype(np.uint8)
    fsm = regex_nfa([(pat, 3)])
    ref, wk = oracle.scan(fsm, x)
    assert len(ref) < 1024
    h = P.pfsm_load(fsm)
    try:
        for seg in (4096, 65536):
            P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, seg)
            n, out = P.pfsm_scan(h, dev(x))
            assert np.array_equal(out.cpu().numpy(), ref), seg
            st = P.pfsm_last_stats(h)
            assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref)), seg
    finally:
        h.free()
