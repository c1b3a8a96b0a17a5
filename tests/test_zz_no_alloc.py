"""The scan entry point that allocates nothing (pfsm_scan_noalloc) against
pfsm_scan_async on the same inputs: equal totals and equal match lists,
element by element, on consecutive calls that share the static scratch."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def both(P, h, x, cap):
    """(total, rows) of pfsm_scan_async and of pfsm_scan_noalloc, in that order."""
    res = []
    for fn in (P.pfsm_scan_async, P.pfsm_scan_noalloc):
        out = torch.full((max(cap, 1), 3), -7, dtype=torch.int32, device="cuda")
        tot = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        fn(h, x, out[:cap], tot)
        torch.cuda.synchronize()
        t = int(tot.item())
        res.append((t, out[:min(t, cap)].cpu().numpy(), out[min(t, cap):].cpu().numpy()))
    return res


def check_pair(P, h, data, cap=None):
    x = dev(data)
    cap = cap if cap is not None else len(data) // 8 + 1024
    (ta, ra, tail_a), (tb, rb, tail_b) = both(P, h, x, cap)
    assert ta == tb, (ta, tb)
    assert ra.shape == rb.shape
    assert np.array_equal(ra, rb)
    # rows past the total (or past cap) are untouched
    assert (tail_b == -7).all()
    return ta, rb


def test_two_calls_second_smaller(P):
    wl = W.cfg2()  # 256-state DFA, 16 MiB
    print(f"noalloc: cfg2 n={len(wl.data)}", flush=True)
    h = P.pfsm_load(wl.automaton)
    try:
        t1, _ = check_pair(P, h, wl.data)
        assert t1 > 100000
        # a ragged, much smaller input on the same scratch, then the oracle
        small = wl.data[:300_001]
        t2, rows = check_pair(P, h, small)
        assert t2 < t1
        ref, _ = oracle.scan(wl.automaton, small)
        assert np.array_equal(rows, ref)
    finally:
        h.free()


def test_other_handle_after_large_call(P):
    wl = W.cfg1()  # 16 states over {a,b,c,d}, 4 KiB
    h = P.pfsm_load(wl.automaton)
    try:
        _, rows = check_pair(P, h, wl.data)
        ref, _ = oracle.scan(wl.automaton, wl.data)
        assert np.array_equal(rows, ref)
        # 10 bytes of the paper's Figure 2 input, as a DFA
        g = P.pfsm_load(subset.to_dfa(W.fig1_nfa()))
        try:
            x = np.frombuffer(W.FIG2_INPUT, np.uint8).copy()
            _, rows = check_pair(P, g, x)
            ref, _ = oracle.scan(subset.to_dfa(W.fig1_nfa()), x)
            assert np.array_equal(rows, ref) and len(ref) == 10
        finally:
            g.free()
    finally:
        h.free()


def test_overflow_and_empty(P):
    wl = W.cfg2(seed=21, n=1 << 20)
    h = P.pfsm_load(wl.automaton)
    try:
        full, _ = check_pair(P, h, wl.data)
        assert full > 1000
        t, rows = check_pair(P, h, wl.data, cap=full // 3)
        assert t == full and len(rows) == full // 3
        t, rows = check_pair(P, h, wl.data[:0], cap=4)
        assert t == 0 and len(rows) == 0
    finally:
        h.free()


def test_limits_rejected_on_the_host(P):
    wl = W.cfg2(seed=5, n=1 << 20)
    h = P.pfsm_load(wl.automaton)
    out = torch.empty((16, 3), dtype=torch.int32, device="cuda")
    tot = torch.zeros(1, dtype=torch.int64, device="cuda")
    try:
        # 16 MiB in 256-byte segments: 65536 segments, past the 32768 held
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, 256)
        big = torch.zeros(16 << 20, dtype=torch.uint8, device="cuda")
        with pytest.raises(P.PfsmError) as e:
            P.pfsm_scan_noalloc(h, big, out, tot)
        assert e.value.code == P.PFSM_EINVAL
    finally:
        h.free()
    nfa = P.pfsm_load(W.fig1_nfa())
    try:
        with pytest.raises(P.PfsmError) as e:
            P.pfsm_scan_noalloc(nfa, dev(np.frombuffer(W.FIG2_INPUT, np.uint8).copy()), out, tot)
        assert e.value.code == P.PFSM_ENOSYS
    finally:
        nfa.free()
