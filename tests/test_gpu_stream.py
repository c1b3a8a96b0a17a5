"""Streaming scans (chained data partitioning, Section III.D.2) against the
oracle: a stream fed in pieces must report, piece by piece, exactly the
oracle's whole-stream matches whose end lies in that piece, in (start, end,
label) order."""
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


def dev(a):
    a = np.array(np.frombuffer(bytes(a), np.uint8)) if isinstance(a, (bytes, bytearray)) else np.array(a, np.uint8)
    return torch.from_numpy(a).cuda()


def feed_pieces(P, fsm, x, cuts, carried=None):
    """Feed x cut at `cuts`; returns [(lo, hi, matches)] and checks, when
    `carried` is given, the live-instance count after every piece."""
    x = np.frombuffer(bytes(x), np.uint8) if isinstance(x, (bytes, bytearray)) else np.asarray(x, np.uint8)
    h = P.pfsm_load(fsm)
    res = []
    try:
        with P.Stream(h) as st:
            lo = 0
            for hi in list(cuts) + [x.size]:
                _, out = st.feed(dev(x[lo:hi]))
                res.append((lo, hi, out.cpu().numpy()))
                pos, car = st.info()
                assert pos == hi
                if carried is not None:
                    assert car == carried(hi), (hi, car)
                lo = hi
    finally:
        h.free()
    return res


def check_stream(P, fsm, x, cuts, carried=None):
    ref, _ = oracle.scan(fsm, x)
    res = feed_pieces(P, fsm, x, cuts, carried)
    for lo, hi, got in res:
        exp = ref[(ref[:, 1] >= lo) & (ref[:, 1] < hi)]
        assert got.shape == exp.shape, (lo, hi, got.shape, exp.shape)
        assert np.array_equal(got, exp), (lo, hi)
    assert sum(len(g) for _, _, g in res) == len(ref)
    return ref


def random_cuts(rng, n, k, align=None):
    c = np.unique(rng.integers(1, n, k))
    if align:
        c = np.unique(np.concatenate([c, (c // align) * align, (c // align) * align + 1]))
        c = c[(c > 0) & (c < n)]
    return [int(v) for v in c]


def test_fig2_byte_by_byte(P):
    ref = check_stream(P, W.fig1_nfa(), W.FIG2_INPUT, list(range(1, len(W.FIG2_INPUT))))
    assert len(ref) == 10


def test_fig2_dfa_form_pieces(P):
    # the same language set through the DFA path (NFA-free walk): literal "ac"
    check_stream(P, W.literal_dfa(b"ac"), W.FIG2_INPUT, [1, 3, 4])


def test_cfg1_pieces(P):
    wl = W.cfg1()
    rng = np.random.default_rng(11)
    check_stream(P, wl.automaton, wl.data, random_cuts(rng, wl.data.size, 25) + [4095])


def test_cfg2_pieces_cut_inside_walks(P):
    wl = W.cfg2(n=1 << 20)
    rng = np.random.default_rng(12)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    # cut inside matches that are at least 3 bytes long, plus random and aligned cuts
    long = ref[ref[:, 1] - ref[:, 0] >= 3]
    inside = [int(s + 1) for s in long[rng.choice(len(long), 12, replace=False), 0]]
    cuts = sorted(set(inside + random_cuts(rng, wl.data.size, 8, align=16)))
    check_stream(P, wl.automaton, wl.data, cuts)


def test_cfg3_pieces(P):
    wl = W.cfg3(n=1 << 20, n_patterns=200, plant_rate=1e-3)
    rng = np.random.default_rng(13)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    long = ref[ref[:, 1] - ref[:, 0] >= 8]
    inside = [int((s + e) // 2) for s, e in long[rng.choice(len(long), 8, replace=False), :2]]
    check_stream(P, wl.automaton, wl.data, sorted(set(inside + random_cuts(rng, wl.data.size, 6))))


def test_sigma_plus_every_start_carried(P):
    # every start stays live: the carried set after k bytes holds k instances
    n = 1500
    x = np.random.default_rng(14).integers(0, 256, n, dtype=np.uint8)
    ref = check_stream(P, W.sigma_plus_dfa(), x, [1, 2, 100, 517, 518, 1024, 1300], carried=lambda k: k)
    assert len(ref) == n * (n + 1) // 2


def test_sigma_plus_many_carried(P):
    # more carried instances than one workgroup sorts in LDS: the
    # device-wide sort path
    n = 4000
    x = np.random.default_rng(17).integers(0, 256, n, dtype=np.uint8)
    ref = check_stream(P, W.sigma_plus_dfa(), x, [2500, 2501, 3999], carried=lambda k: k)
    assert len(ref) == n * (n + 1) // 2


def test_many_carried_merge_passes(P):
    # 30,000 live starts at the cut: 15 sorted tiles (the last ragged) and
    # four merge passes before the carried set is compacted
    from oracle import subset
    rng = np.random.default_rng(18)
    fsm = subset.to_dfa(regex_nfa([(b"[a-d]+e", 0)]))
    abcd = np.frombuffer(b"abcd", np.uint8)
    x = np.concatenate([rng.choice(abcd, 30000), np.frombuffer(b"eabce", np.uint8), rng.choice(abcd, 100)])
    ref = check_stream(P, fsm, x, [30000, 30002])
    assert len(ref) == 30003


def test_many_carried_nfa_sets(P):
    # every start carries several NFA states (and repeated pairs): 6,000
    # starts whose sets go through the tile sort, the merges and the
    # de-duplication
    rng = np.random.default_rng(19)
    nfa = regex_nfa([(b"[a-d]*e", 0), (b"[a-d]*ae", 1), (b"[a-c]*de", 2), (b"[a-d][a-d]*f", 3)])
    abcd = np.frombuffer(b"abcd", np.uint8)
    x = np.concatenate([rng.choice(abcd, 6000), np.frombuffer(b"aefde", np.uint8), rng.choice(abcd, 50)])
    ref = check_stream(P, nfa, x, [6000, 6001, 6003], carried=None)
    assert len(ref) > 12000


def test_sigma_plus_nfa_every_start_carried(P):
    n = 700
    x = np.random.default_rng(15).integers(0, 256, n, dtype=np.uint8)
    ref = check_stream(P, W.dfa_as_nfa(W.sigma_plus_dfa()), x, [5, 300, 301, 650], carried=lambda k: k)
    assert len(ref) == n * (n + 1) // 2


def test_large_sets_cross_pieces(P):
    # unions whose sets exceed what a lane keeps: the workgroup replay path
    # reaches the end of a piece and hands its frontier on
    pats = [(b"[a-d]*a", 0), (b"[a-d]*b", 1), (b"[a-d]*c[a-d]", 2), (b"[ab]*dd", 3), (b"(a|c)*b[a-d]", 4),
            (b"[a-d]*ab", 5), (b"[cd]*a", 6)]
    rng = np.random.default_rng(16)
    x = bytes(rng.choice(list(b"abcd"), 400).astype(np.uint8))
    check_stream(P, regex_nfa(pats), x, [1, 50, 51, 64, 200, 399])


@pytest.mark.parametrize("seed", range(6))
def test_random_dfas(P, seed):
    rng = np.random.default_rng(100 + seed)
    fsm = W.random_dfa(rng, 12, 4, p_dead=0.3, n_finals=3)
    x = bytes(rng.choice(list(b"abcde"), 3000).astype(np.uint8))
    check_stream(P, fsm, x, random_cuts(rng, len(x), 10))


@pytest.mark.parametrize("seed", range(6))
def test_random_nfas(P, seed):
    rng = np.random.default_rng(200 + seed)
    fsm = W.random_nfa(rng, 14, list(b"abcd"), 30)
    x = bytes(rng.choice(list(b"abcde"), 800).astype(np.uint8))
    check_stream(P, fsm, x, random_cuts(rng, len(x), 10))


def test_overflow_leaves_stream_unchanged(P):
    wl = W.cfg1()
    x = wl.data
    ref, _ = oracle.scan(wl.automaton, x)
    h = P.pfsm_load(wl.automaton)
    try:
        with P.Stream(h) as st:
            _, a = st.feed(dev(x[:1000]))
            piece = dev(x[1000:3000])
            want = ref[(ref[:, 1] >= 1000) & (ref[:, 1] < 3000)]
            assert len(want) > 1
            small = torch.empty((1, 3), dtype=torch.int32, device="cuda")
            with pytest.raises(P.PfsmError) as e:
                st.feed(piece, out=small)
            assert e.value.code == P.PFSM_EOVERFLOW
            assert st.info()[0] == 1000
            _, b = st.feed(piece)
            _, c = st.feed(dev(x[3000:]))
        got = np.concatenate([a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()])
        assert np.array_equal(b.cpu().numpy(), want)
        assert np.array_equal(np.unique(got, axis=0), ref)
    finally:
        h.free()


def test_empty_piece_and_edit_guard(P):
    fsm = regex_nfa([(b"ab+c", 0), (b"b+", 1)])
    h = P.pfsm_load(fsm)
    try:
        with P.Stream(h) as st:
            st.feed(dev(b"aab"))
            before = st.info()
            n, _ = st.feed(dev(b""))
            assert n == 0 and st.info() == before
            n, out = st.feed(dev(b"bc"))
            ref, _ = oracle.scan(fsm, b"aabbc")
            assert np.array_equal(out.cpu().numpy(), ref[ref[:, 1] >= 3])
            P.pfsm_add_pattern(h, regex_nfa([(b"c", 7)]))
            with pytest.raises(P.PfsmError) as e:
                st.feed(dev(b"c"))
            assert e.value.code == P.PFSM_EINVAL
    finally:
        h.free()
