"""Tag-merged DFA stepping (Section III.B tag sets) against the oracle: the
same matches, bit for bit, and the same work counters (instance-steps and
live steps, counted per instance although the kernel steps per state)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1110_1716_amd as P
    P.load_library()
    return P


def dev(a, offset=0):
    a = np.asarray(a, np.uint8)
    buf = torch.zeros(a.size + offset, dtype=torch.uint8)
    buf[offset:] = torch.from_numpy(a.copy())
    return buf.cuda()[offset:]


def check_merged(P, fsm, x, offset=0):
    x = np.frombuffer(bytes(x), np.uint8) if isinstance(x, (bytes, bytearray)) else np.asarray(x, np.uint8)
    ref, wk = oracle.scan(fsm, x)
    h = P.pfsm_load(fsm)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_MERGED_WALKS, 1)
        n, out = P.pfsm_scan(h, dev(x, offset))
        got = out.cpu().numpy()
        assert got.shape == ref.shape, (got.shape, ref.shape)
        assert np.array_equal(got, ref)
        if x.size:
            st = P.pfsm_last_stats(h)
            assert st["transitions"] == wk["T"]
            assert st["activations"] == wk["X"]
            assert st["matches"] == len(ref)
    finally:
        h.free()
    return ref


def test_log_search(P):
    wl = W.log_search(n=256 << 10, line_mean=512)
    ref = check_merged(P, wl.automaton, wl.data)
    assert len(ref) > 1000


@pytest.mark.parametrize("seed", [1, 100, 101, 102, 103])
def test_cfg1_family(P, seed):
    wl = W.cfg1(seed=seed, n=8192)
    check_merged(P, wl.automaton, wl.data)


def test_sigma_plus(P):
    n = 3000
    x = np.random.default_rng(3).integers(0, 256, n, dtype=np.uint8)
    ref = check_merged(P, W.sigma_plus_dfa(labels=(0, 5)), x)
    assert len(ref) == n * (n + 1)


@pytest.mark.parametrize("n", [1, 15, 17, 1023, 1024, 1025, 4097, 70001])
def test_ragged_sizes(P, n):
    rng = np.random.default_rng(n)
    fsm = W.random_dfa(rng, 10, 4, p_dead=0.2, n_finals=3, max_labels=3)
    x = rng.choice(list(b"abcde"), n).astype(np.uint8)
    check_merged(P, fsm, x, offset=n % 16)


@pytest.mark.parametrize("seed", range(6))
def test_random_dfas(P, seed):
    rng = np.random.default_rng(300 + seed)
    n_states = int(rng.integers(2, 64))
    fsm = W.random_dfa(rng, n_states, 5, p_dead=float(rng.uniform(0.0, 0.5)), n_finals=3, max_labels=2)
    x = rng.choice(list(b"abcdef"), 20000).astype(np.uint8)
    check_merged(P, fsm, x, offset=seed)


def test_max_states_all_active(P):
    # 63 states, few dead transitions: up to 63 distinct states live at once
    rng = W.rng_for(77)
    d = W.random_table_dfa(rng, 63, 256, 0.02, 4)
    x = rng.integers(0, 256, 50000, dtype=np.uint8)
    check_merged(P, d, x)


def test_merged_option_errors(P):
    big = W.random_table_dfa(W.rng_for(5), 64, 256, 0.5, 2)
    for fsm in (W.fig1_nfa(), big):
        h = P.pfsm_load(fsm)
        try:
            with pytest.raises(P.PfsmError) as e:
                P.pfsm_set_option(h, P.PFSM_OPT_MERGED_WALKS, 1)
            assert e.value.code == P.PFSM_ENOSYS
        finally:
            h.free()


def test_tuner_picks_merged_for_long_walks(P):
    wl = W.log_search(n=1 << 20, line_mean=1024)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        x = dev(wl.data)
        rep = P.pfsm_tune(h, x, reps=2)
        assert rep["merged_walks"] == 1, rep
        assert rep["ms_after"] < rep["ms_before"]
        n, out = P.pfsm_scan(h, x)
        assert np.array_equal(out.cpu().numpy(), ref)
    finally:
        h.free()


@pytest.mark.parametrize("limit", [1, 3, 40])
def test_count_limit_memory_paths(P, limit):
    # a small 32-bit limit moves per-start counts to memory during the count
    # walk and keeps whole segments' offsets there during the write walk;
    # matches and work counters stay those of the oracle
    cases = [(W.log_search(n=256 << 10, line_mean=512).automaton, W.log_search(n=256 << 10, line_mean=512).data),
             (W.sigma_plus_dfa(labels=(0, 5)), np.random.default_rng(3).integers(0, 256, 3000, dtype=np.uint8))]
    for fsm, x in cases:
        ref, wk = oracle.scan(fsm, x)
        h = P.pfsm_load(fsm)
        try:
            P.pfsm_set_option(h, P.PFSM_OPT_MERGED_WALKS, 1)
            P.pfsm_set_option(h, P.PFSM_OPT_MERGED_COUNT_LIMIT, limit)
            assert P.pfsm_get_option(h, P.PFSM_OPT_MERGED_COUNT_LIMIT) == limit
            n, out = P.pfsm_scan(h, dev(x))
            assert np.array_equal(out.cpu().numpy(), ref)
            st = P.pfsm_last_stats(h)
            assert (st["transitions"], st["activations"], st["matches"]) == (wk["T"], wk["X"], len(ref))
        finally:
            h.free()
