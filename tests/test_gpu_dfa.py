"""GPU parity of the DFA scan against the CPU oracle (bit-exact match lists)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import subset

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
    return torch.from_numpy(np.array(np.frombuffer(bytes(x), np.uint8)
                                                 if isinstance(x, (bytes, bytearray)) else x)).cuda()


def gpu_scan(P, fsm, x, **kw):
    h = P.pfsm_load(fsm)
    try:
        n, out = P.pfsm_scan(h, dev(x), **kw)
        stats = P.pfsm_last_stats(h) if len(x) else None
        return out.cpu().numpy(), stats
    finally:
        h.free()


def check(P, fsm, x, work=True):
    ref, wk = oracle.scan(fsm, x)
    got, stats = gpu_scan(P, fsm, x)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.array_equal(got, ref)
    if work and stats is not None:
        assert stats["transitions"] == wk["T"]
        assert stats["activations"] == wk["X"]
        assert stats["matches"] == len(ref)
    return ref


def test_fig2_as_dfa(P):
    ref = check(P, subset.to_dfa(W.fig1_nfa()), W.FIG2_INPUT)
    assert len(ref) == 10


def test_cfg1_full(P):
    wl = W.cfg1()
    check(P, wl.automaton, wl.data)


@pytest.mark.parametrize("n_states, p_dead", [(3, 0.2), (254, 0.5), (255, 0.5), (255, 0.9), (256, 0.5), (256, 0.9)])
def test_byte_tables_at_the_8bit_boundary(P, n_states, p_dead):
    # Byte-wide tables of at most 255 states store "no transition" as 255,
    # one past the last state at 255 states; 256 states keep a dead bit per
    # entry.  Walks of every length over a ragged input: matches, T and X.
    rng = np.random.default_rng(1000 + n_states + int(100 * p_dead))
    fsm = W.random_table_dfa(rng, n_states, 256, p_dead, min(n_states - 1, 8))
    x = rng.integers(0, 256, 70001, dtype=np.uint8)
    ref = check(P, fsm, x)
    assert len(ref) > 0


@pytest.mark.parametrize("seed", [2, 21])
def test_cfg2_full(P, seed):
    wl = W.cfg2(seed=seed)
    ref = check(P, wl.automaton, wl.data)
    assert len(ref) > 100000


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 1000, 4095, 4096, 4097, 4352, 70001, 1 << 20])
def test_ragged_sizes(P, n):
    wl = W.cfg2(seed=5, n=n, plant_every=max(n, 64)) if n >= 64 else W.cfg2(seed=5, n=64, plant_every=64)
    x = wl.data[:n]
    check(P, wl.automaton, x)


@pytest.mark.parametrize("offset", [1, 3, 7, 13])
def test_unaligned_input(P, offset):
    wl = W.cfg2(seed=6, n=1 << 16)
    ref, _ = oracle.scan(wl.automaton, wl.data[offset:])
    h = P.pfsm_load(wl.automaton)
    xd = dev(wl.data)[offset:]
    n, out = P.pfsm_scan(h, xd)
    h.free()
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_dfas(P, seed):
    rng = np.random.default_rng(500 + seed)
    d = W.random_dfa(rng, int(rng.integers(1, 40)), int(rng.integers(1, 6)), p_dead=0.3,
                     n_finals=int(rng.integers(1, 5)), max_labels=3, n_labels=5)
    x = bytes(rng.choice(list(b"abcdefg"), int(rng.integers(1, 6000))).astype(np.uint8))
    check(P, d, x)


def test_sigma_plus_dense_windows(P):
    """Every substring matches: every window overflows its LDS match buffer."""
    n = 3000
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    ref = check(P, W.sigma_plus_dfa((2, 0)), x)
    assert len(ref) == 2 * n * (n + 1) // 2


def test_overflow_reports_exact_count_and_prefix(P):
    wl = W.cfg2(seed=7, n=1 << 18)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    h = P.pfsm_load(wl.automaton)
    out = torch.empty((100, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(P.PfsmError) as ei:
        P.pfsm_scan(h, dev(wl.data), out=out)
    assert ei.value.code == P.PFSM_EOVERFLOW
    assert np.array_equal(out.cpu().numpy(), ref[:100])
    n, out2 = P.pfsm_scan(h, dev(wl.data))  # automatic growth
    assert n == len(ref) and np.array_equal(out2.cpu().numpy(), ref)
    h.free()


def test_empty_input(P):
    h = P.pfsm_load(W.cfg1().automaton)
    n, out = P.pfsm_scan(h, torch.empty(0, dtype=torch.uint8, device="cuda"))
    assert n == 0
    cnt = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    P.pfsm_scan_async(h, torch.empty(0, dtype=torch.uint8, device="cuda"),
                      torch.empty((1, 3), dtype=torch.int32, device="cuda"), cnt)
    assert int(cnt.item()) == 0
    h.free()


def test_back_to_back_async_scans_reset_their_state(P):
    """Consecutive launches on one stream reuse the workspace (tickets, status words)."""
    wl = W.cfg2(seed=9, n=3 << 20)
    h = P.pfsm_load(wl.automaton)
    sizes = [3 << 20, 5000, 1 << 20, 123457, 3 << 20]
    xs = [dev(wl.data[:s]) for s in sizes]
    outs = [torch.empty((s // 16 + 1024, 3), dtype=torch.int32, device="cuda") for s in sizes]
    cnts = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    for i in range(len(sizes)):
        P.pfsm_scan_async(h, xs[i], outs[i], cnts[i:i + 1])
    torch.cuda.synchronize()
    for i, s in enumerate(sizes):
        ref, _ = oracle.scan(wl.automaton, wl.data[:s])
        c = int(cnts[i].item())
        assert c == len(ref)
        assert np.array_equal(outs[i][:c].cpu().numpy(), ref)
    h.free()


def test_remove_label_disables_it(P):
    wl = W.cfg2(seed=10, n=1 << 20)
    full, _ = oracle.scan(wl.automaton, wl.data)
    h = P.pfsm_load(wl.automaton)
    P.pfsm_remove_pattern(h, 3)
    n, out = P.pfsm_scan(h, dev(wl.data))
    assert np.array_equal(out.cpu().numpy(), full[full[:, 2] != 3])
    with pytest.raises(P.PfsmError) as ei:
        P.pfsm_remove_pattern(h, 3)
    assert ei.value.code == P.PFSM_ENOENT
    with pytest.raises(P.PfsmError) as ei:
        P.pfsm_add_pattern(h, W.fig1_nfa())
    assert ei.value.code == P.PFSM_ENOSYS
    h.free()


def test_deterministic(P):
    wl = W.cfg2(seed=11, n=1 << 22)
    h = P.pfsm_load(wl.automaton)
    x = dev(wl.data)
    a = P.pfsm_scan(h, x)[1].cpu().numpy()
    b = P.pfsm_scan(h, x)[1].cpu().numpy()
    h.free()
    assert np.array_equal(a, b)


def test_invalid_descriptors_rejected(P):
    d = W.literal_dfa(b"abc")
    bad = W.DFA(d.n_states, d.n_symbols, d.q0, None, d.delta.copy(), d.final_off, d.final_labels)
    bad.delta[5] = 1000
    with pytest.raises(P.PfsmError) as ei:
        P.pfsm_load(bad)
    assert ei.value.code == P.PFSM_EINVAL
    bad2 = W.DFA(d.n_states, 200, d.q0, None, d.delta[:200 * d.n_states], d.final_off, d.final_labels)
    with pytest.raises(P.PfsmError):
        P.pfsm_load(bad2)


def test_dropped_walks_recounted(P):
    # every start lives to the end of its line: with 64 KiB segments the
    # parked walks outgrow the spill area, the segment falls back to fresh
    # per-start walks, and its count and work must still be exact
    wl = W.log_search(n=256 << 10, line_mean=512)
    ref, wk = oracle.scan(wl.automaton, wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, 65536)
        n, out = P.pfsm_scan(h, dev(wl.data))
        assert np.array_equal(out.cpu().numpy(), ref)
        st = P.pfsm_last_stats(h)
        assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref))
    finally:
        h.free()


def one_byte_dfa():
    """Two states: q0 -> q1 (final, label 4) on bytes < 128, nothing else:
    one match (i, i, 4) at every position holding such a byte."""
    delta = -np.ones(2 * 256, dtype=np.int32)
    delta[:128] = 1
    off, lab = W.label_csr(2, {1: [4]})
    return W.DFA(2, 256, 0, None, delta, off, lab)


@pytest.mark.parametrize("n, seg", [(2 << 20, 256), (1 << 20, 0)])
def test_deferred_placement_launch_paths(P, n, seg):
    # 8,192 segments of 256 B (two follow-up launches) and the automatic
    # segments (one fused launch): bit-exact rows and exact counts
    wl = W.cfg2(seed=21, n=n)
    ref, wk = oracle.scan(wl.automaton, wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, seg)
        k, out = P.pfsm_scan(h, dev(wl.data))
        assert np.array_equal(out.cpu().numpy(), ref)
        st = P.pfsm_last_stats(h)
        assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref))
        # an output too small: the count is still exact, and the output
        # holds the first cap matches
        cap = len(ref) // 3
        small = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        P.pfsm_scan_async(h, dev(wl.data), small, cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == len(ref)
        assert np.array_equal(small.cpu().numpy(), ref[:cap])
        # and the next scan on the stream is whole again
        k2, out2 = P.pfsm_scan(h, dev(wl.data))
        assert np.array_equal(out2.cpu().numpy(), ref)
    finally:
        h.free()


def test_deferred_staging_full(P):
    # about 4.7 M matches in 9,216 segments of 1 KiB that each fit their LDS
    # buffer: the staging rows run out part way, and the remaining segments
    # are placed by the scan itself
    rng = np.random.default_rng(22)
    x = rng.integers(0, 256, 9 << 20, dtype=np.uint8)
    fsm = one_byte_dfa()
    ref, wk = oracle.scan(fsm, x)
    assert len(ref) > (4 << 20) + (256 << 10)
    h = P.pfsm_load(fsm)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, 1024)
        for _ in range(2):
            k, out = P.pfsm_scan(h, dev(x), cap=len(ref))
            assert k == len(ref)
            assert np.array_equal(out.cpu().numpy(), ref)
    finally:
        h.free()
