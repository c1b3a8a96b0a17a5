"""Seeded parity sweep: random DFAs and NFAs of every table encoding, input
lengths that cross slice, window and segment boundaries, unaligned inputs,
and the launch settings a handle accepts; and DFA scans of 256 KiB-4 MiB
with automatic segments.  Each case must reproduce the oracle's match list
bit for bit and its work counters (instance-steps, live steps, matches)."""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.regex import regex_nfa

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PATTERNS = [b"a.{0,3}b", b"(ab|cd)+", b"a(b|c)*d", b"[a-c]+d?", b"(a|b)*abb", b"d{2,}", b"a*c", b"((a|b)(c|d))+"]


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1110_1716_amd as P
    P.load_library()
    return P


def dev(a, offset):
    buf = torch.zeros(a.size + offset, dtype=torch.uint8)
    buf[offset:] = torch.from_numpy(a.copy())
    return buf.cuda()[offset:]


def make_case(seed):
    """(automaton, input bytes, options) for one seed; inputs stay small
    where walks are long, so that the oracle and the output stay small."""
    rng = np.random.default_rng(7000 + seed)
    kind = seed % 4
    opts = {"segment": int(rng.choice([0, 256, 1024, 4096, 65536]))}
    if kind == 0:
        p_dead = float(rng.uniform(0.05, 0.7))
        fsm = W.random_dfa(rng, int(rng.integers(2, 60)), 4, p_dead=p_dead, n_finals=int(rng.integers(1, 4)),
                           max_labels=3, n_labels=5)
        n = int(rng.choice([1, 15, 17, 1000, 1025, 3000] + ([4097, 12288] if p_dead > 0.4 else [])))
        alphabet = list(b"abcd")
        if rng.random() < 0.5:
            opts["merged"] = 1
    elif kind == 1:
        n_states = int(rng.choice([40, 200, 256, 300, 1000]))
        fsm = W.random_table_dfa(rng, n_states, 256, float(rng.uniform(0.85, 0.97)), int(rng.integers(1, 17)))
        n = int(rng.choice([255, 1024, 4095, 4097, 20000, 40000]))
        alphabet = list(range(256))
        if n_states <= 63 and rng.random() < 0.5:
            opts["merged"] = 1
    elif kind == 2:
        k = int(rng.integers(2, 14))
        fsm = W.random_nfa(rng, k, list(b"abc"), n_edges=int(rng.integers(k, 3 * k)), p_eps=0.2,
                           n_finals=int(rng.integers(1, 4)))
        n = int(rng.choice([1, 17, 1000, 4097, 6000]))
        alphabet = list(b"abcd")
        opts["pair"] = int(rng.integers(0, 2))
    else:
        pats = [(PATTERNS[int(j)], i) for i, j in enumerate(rng.choice(len(PATTERNS), int(rng.integers(1, 4)),
                                                                       replace=False))]
        fsm = regex_nfa(pats)
        n = int(rng.choice([1, 500, 3000, 4097, 6000]))
        alphabet = list(b"abcd")
        opts["pair"] = int(rng.integers(0, 2))
    x = rng.choice(alphabet, n).astype(np.uint8)
    x[rng.random(n) < 0.02] = ord("e")  # a byte outside the small alphabets
    return fsm, x, int(rng.integers(0, 16)), opts


@pytest.mark.parametrize("seed", range(160))
def test_sweep(P, seed):
    fsm, x, offset, opts = make_case(seed)
    ref, wk = oracle.scan(fsm, x)
    h = P.pfsm_load(fsm)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, opts["segment"])
        if opts.get("merged"):
            try:
                P.pfsm_set_option(h, P.PFSM_OPT_MERGED_WALKS, 1)
            except P.PfsmError as e:
                assert e.code == P.PFSM_ENOSYS
        if "pair" in opts:
            P.pfsm_set_option(h, P.PFSM_OPT_PAIR_CACHE, opts["pair"])
        n, out = P.pfsm_scan(h, dev(x, offset))
        got = out.cpu().numpy()
        assert got.shape == ref.shape, (got.shape, ref.shape, opts)
        assert np.array_equal(got, ref), opts
        if x.size:
            st = P.pfsm_last_stats(h)
            assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref)), opts
    finally:
        h.free()


def tiled(x, n):
    """n bytes of x repeated (x non-empty)."""
    return np.tile(x, -(-n // x.size))[:n] if n else np.zeros(0, np.uint8)


@pytest.mark.parametrize("seed", range(16))
def test_sweep_batch(P, seed):
    # 2-4 automata of the cases above, 3-30 streams of mixed lengths, one launch
    rng = np.random.default_rng(9000 + seed)
    cases = [make_case(int(s)) for s in rng.choice(160, int(rng.integers(2, 5)), replace=False)]
    autos = [c[0] for c in cases]
    aut_of = rng.integers(0, len(autos), int(rng.integers(3, 31))).astype(np.int32)
    streams = [tiled(cases[a][1], int(rng.choice([0, 1, 15, 17, 700, 4097, 9000]))) if cases[a][1].size
               else np.zeros(0, np.uint8) for a in aut_of]
    off = np.zeros(len(streams) + 1, np.int64)
    off[1:] = np.cumsum([s.size for s in streams])
    data = np.concatenate(streams + [np.zeros(16, np.uint8)])
    hs = [P.pfsm_load(a) for a in autos]
    try:
        n, got, mo = P.pfsm_scan_batch(hs, torch.from_numpy(data).cuda(), torch.from_numpy(off).cuda(),
                                       torch.from_numpy(aut_of).cuda())
        got, mo = got.cpu().numpy(), mo.cpu().numpy()
    finally:
        for h in hs:
            h.free()
    assert mo[0] == 0 and mo[-1] == n == len(got)
    for i, x in enumerate(streams):
        ref, _ = oracle.scan(autos[aut_of[i]], x)
        assert np.array_equal(got[mo[i]:mo[i + 1]], ref), (i, x.size)


@pytest.mark.parametrize("seed", range(24))
def test_sweep_stream(P, seed):
    # one case fed in random pieces: each feed reports the matches ending in
    # its piece, in the whole scan's order
    fsm, x, _, _ = make_case((7 * seed) % 160)
    rng = np.random.default_rng(9500 + seed)
    ref, _ = oracle.scan(fsm, x)
    cuts = sorted(set(int(c) for c in rng.integers(1, x.size, int(rng.integers(1, 12))))) if x.size > 1 else []
    h = P.pfsm_load(fsm)
    total = 0
    try:
        with P.Stream(h) as st:
            lo = 0
            for hi in cuts + [x.size]:
                _, out = st.feed(torch.from_numpy(x[lo:hi].copy()).cuda())
                exp = ref[(ref[:, 1] >= lo) & (ref[:, 1] < hi)]
                assert np.array_equal(out.cpu().numpy(), exp), (lo, hi)
                total += len(exp)
                lo = hi
    finally:
        h.free()
    assert total == len(ref)


def make_large_case(seed):
    """DFA scans of 256 KiB-4 MiB with automatic segments: enough segments
    for plain scans to stage their matches and place them afterwards."""
    rng = np.random.default_rng(50000 + seed)
    kind = seed % 3
    n = int(rng.choice([256 << 10, 300001, 1 << 20, 2 << 20, 4 << 20]))
    if kind == 0:
        ns = int(rng.choice([16, 64, 256, 1000]))
        fsm = W.random_table_dfa(rng, ns, 256, float(rng.uniform(0.85, 0.97)),
                                 int(rng.integers(1, min(17, ns // 4 + 1))))
        x = rng.integers(0, 256, n, dtype=np.uint8)
    elif kind == 1:
        fsm = W.random_dfa(rng, int(rng.integers(2, 60)), 4, p_dead=float(rng.uniform(0.45, 0.8)),
                           n_finals=int(rng.integers(1, 4)), max_labels=3, n_labels=5)
        x = (rng.integers(0, 4, n) + ord("a")).astype(np.uint8)
        x[rng.random(n) < 0.02] = ord("e")
    else:
        wl = W.cfg2(seed=int(rng.integers(0, 1 << 30)), n=n)
        fsm, x = wl.automaton, wl.data
    return fsm, x


@pytest.mark.parametrize("seed", range(60))
def test_sweep_large(P, seed):
    fsm, x = make_large_case(seed)
    ref, wk = oracle.scan(fsm, x)
    h = P.pfsm_load(fsm)
    try:
        n, out = P.pfsm_scan(h, torch.from_numpy(x).cuda())
        assert np.array_equal(out.cpu().numpy(), ref)
        st = P.pfsm_last_stats(h)
        assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref))
    finally:
        h.free()
