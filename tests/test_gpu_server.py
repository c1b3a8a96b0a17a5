"""GPU tests of the continuous-batching server (pfsm_server_*): every result
equals the oracle's and the same request's result when it runs alone."""
import threading

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


def automata():
    return [W.cfg1(seed=5).automaton, W.cfg1(seed=6).automaton,
            W.cfg3(seed=9, n=1 << 16, n_patterns=120).automaton,
            W.cfg3(seed=10, n=1 << 16, n_patterns=80).automaton]


def request_bytes(rng, a, n, perm):
    if a < 2:
        return (rng.integers(0, 4, n) + ord("a")).astype(np.uint8)
    return W.zipf_bytes(rng, n, perm=perm)


def test_alone_equals_mixed_and_oracle(P):
    autos = automata()
    hs = [P.pfsm_load(a) for a in autos]
    rng = np.random.default_rng(7)
    perm = rng.permutation(256).astype(np.uint8)
    probe = [(0, request_bytes(rng, 0, 3000, perm)), (2, request_bytes(rng, 2, 70000, perm)),
             (3, request_bytes(rng, 3, 5, perm))]
    mix = []
    for _ in range(60):
        a = int(rng.integers(0, 4))
        n = int(np.exp(rng.uniform(np.log(1), np.log(200000))))
        mix.append((a, request_bytes(rng, a, n, perm)))
    with P.Server(hs, mem_budget=8 << 20, max_batch=32) as sv:
        alone = [sv.wait(sv.submit(a, x)) for a, x in probe]
        ids = []
        for k, (a, x) in enumerate(mix):
            ids.append(sv.submit(a, x))
            if k % 20 == 10:
                for a2, x2 in probe:
                    ids.append(sv.submit(a2, x2))
        res = [sv.wait(i) for i in ids]
        st = sv.stats()
    reqs = []
    for k, item in enumerate(mix):
        reqs.append(item)
        if k % 20 == 10:
            reqs.extend(probe)
    for (a, x), got in zip(reqs, res):
        ref, _ = oracle.scan(autos[a], x)
        assert np.array_equal(got, ref)
    for (a, x), got in zip(probe, alone):
        ref, _ = oracle.scan(autos[a], x)
        assert np.array_equal(got, ref)
    assert st["requests"] == len(ids) + len(probe)
    assert st["batches"] < st["requests"]  # requests were batched together
    for h in hs:
        h.free()


def test_budget_smaller_than_a_request(P):
    autos = automata()[:1]
    hs = [P.pfsm_load(a) for a in autos]
    rng = np.random.default_rng(8)
    x = (rng.integers(0, 4, 100000) + ord("a")).astype(np.uint8)
    with P.Server(hs, mem_budget=1000, max_batch=4) as sv:
        got = [sv.wait(sv.submit(0, x)) for _ in range(2)]
    ref, _ = oracle.scan(autos[0], x)
    assert all(np.array_equal(g, ref) for g in got)
    hs[0].free()


def test_output_larger_than_estimate_reruns(P):
    d = W.sigma_plus_dfa((1,))
    h = P.pfsm_load(d)
    x = np.random.default_rng(9).integers(0, 256, 2000, dtype=np.uint8)
    with P.Server([h], mem_budget=1 << 28) as sv:
        got = sv.wait(sv.submit(0, x))
        st = sv.stats()
    ref, _ = oracle.scan(d, x)
    assert len(ref) == 2000 * 2001 // 2
    assert np.array_equal(got, ref)
    assert st["reruns"] >= 1
    h.free()


def test_concurrent_submitters(P):
    autos = automata()
    hs = [P.pfsm_load(a) for a in autos]
    rng = np.random.default_rng(10)
    perm = rng.permutation(256).astype(np.uint8)
    work = [[(int(a), request_bytes(rng, int(a), int(rng.integers(1, 50000)), perm))
             for a in rng.integers(0, 4, 15)] for _ in range(4)]
    results = [None] * 4
    with P.Server(hs, mem_budget=4 << 20, max_batch=16) as sv:
        def client(t):
            results[t] = [sv.wait(sv.submit(a, x)) for a, x in work[t]]
        th = [threading.Thread(target=client, args=(t,)) for t in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    for t in range(4):
        for (a, x), got in zip(work[t], results[t]):
            ref, _ = oracle.scan(autos[a], x)
            assert np.array_equal(got, ref)
    for h in hs:
        h.free()


def test_bad_automaton(P):
    hs = [P.pfsm_load(W.cfg1(seed=5).automaton)]
    with P.Server(hs) as sv:
        with pytest.raises(P.PfsmError) as ei:
            sv.submit(3, b"abc")
        assert ei.value.code == P.PFSM_EINVAL
    hs[0].free()


def test_wait_then_release_and_empty_results(P):
    # results stay readable across waits until release; a request with no
    # matches and an empty request give empty results; release twice fails
    autos = automata()[:1]
    hs = [P.pfsm_load(a) for a in autos]
    rng = np.random.default_rng(11)
    x = (rng.integers(0, 4, 50000) + ord("a")).astype(np.uint8)
    ref, _ = oracle.scan(autos[0], x)
    assert len(ref) > 0
    none = np.full(4000, ord("z"), np.uint8)  # a byte outside the alphabet: no match
    with P.Server(hs, mem_budget=64 << 20, max_batch=8) as sv:
        ids = [sv.submit(0, y) for _ in range(3) for y in (x, none, np.zeros(0, np.uint8))]
        for i in ids:
            first = sv.wait(i, release=False)
            again = sv.wait(i, release=False)
            assert np.array_equal(first, again)
            t_sub, t_done = sv.times(i)
            assert t_done >= t_sub > 0
            sv.release(i)
            with pytest.raises(P.PfsmError) as ei:
                sv.release(i)
            assert ei.value.code == P.PFSM_ENOENT
        got = [sv.wait(sv.submit(0, y)) for y in (x, none)]
    assert np.array_equal(got[0], ref)
    assert got[1].shape == (0, 3)
    for h in hs:
        h.free()


def test_held_results_survive_later_batches(P):
    # requests of one batch share its pinned result rows: a result held past
    # the release of its batch-mates and across later batches (which recycle
    # released result buffers) still reads as the oracle's
    w3 = W.cfg3(seed=21, n=1 << 16, n_patterns=120, plant_rate=2e-3)
    autos = [W.cfg1(seed=5).automaton, w3.automaton]
    hs = [P.pfsm_load(a) for a in autos]
    rng = np.random.default_rng(12)

    def req(a):
        n = int(rng.integers(2000, 30000))
        if a == 0:
            return (rng.integers(0, 4, n) + ord("a")).astype(np.uint8)
        o = int(rng.integers(0, w3.data.size - n))
        return np.ascontiguousarray(w3.data[o:o + n])

    first = [(a, req(a)) for a in (0, 1, 0, 1, 0, 1)]
    with P.Server(hs, mem_budget=64 << 20, max_batch=8) as sv:
        ids = [sv.submit(a, x) for a, x in first]
        reads = [sv.wait(i, release=False) for i in ids]
        held = ids[::2] + ids[1:2]
        for i in ids[3::2]:
            sv.release(i)
        for _ in range(4):
            more = [(int(a), req(int(a))) for a in rng.integers(0, 2, 6)]
            got = [sv.wait(i) for i in [sv.submit(a, x) for a, x in more]]
            for (a, x), g in zip(more, got):
                assert np.array_equal(g, oracle.scan(autos[a], x)[0])
        again = [sv.wait(i, release=False) for i in held]
        for i in held:
            sv.release(i)
    for (a, x), got in zip(first, reads):
        ref, _ = oracle.scan(autos[a], x)
        assert len(ref) > 0
        assert np.array_equal(got, ref)
    for i, g in zip(held, again):
        assert np.array_equal(g, reads[ids.index(i)])
    for h in hs:
        h.free()


def test_cfg5_full_size_alone_equals_mixed(P):
    """The served workload at its stated size: 8 resident automata (4 random
    16-state DFAs, 4 NFA unions of 2,000 signatures) and requests log-uniform
    on 256 B-4 MiB.  Probe requests served alone, then mixed among the others
    while they run: every result equals the oracle's."""
    wl = W.cfg5()
    hs = [P.pfsm_load(a) for a in wl.automata]
    rng = np.random.default_rng(55)
    reqs = wl.requests(rng, 120)
    # probes: the largest request of each automaton present
    probe = []
    for a in range(len(wl.automata)):
        mine = [x for b, x in reqs if b == a]
        if mine:
            probe.append((a, max(mine, key=len)))
    print(f"cfg5 full: {len(reqs)} requests, {sum(len(x) for _, x in reqs)} bytes, "
          f"largest {max(len(x) for _, x in reqs)}", flush=True)
    try:
        with P.Server(hs, mem_budget=1 << 30, max_batch=256) as sv:
            alone = [sv.wait(sv.submit(a, x, borrow=True)) for a, x in probe]
            ids, order = [], []
            for k, (a, x) in enumerate(reqs):
                ids.append(sv.submit(a, x, borrow=True))
                order.append((a, x))
                if k % 30 == 15:
                    for a2, x2 in probe:
                        ids.append(sv.submit(a2, x2, borrow=True))
                        order.append((a2, x2))
            mixed = [sv.wait(i) for i in ids]
        for (a, x), got in zip(order, mixed):
            ref, _ = oracle.scan(wl.automata[a], x)
            assert np.array_equal(got, ref), (a, len(x))
        for (a, x), got in zip(probe, alone):
            ref, _ = oracle.scan(wl.automata[a], x)
            assert np.array_equal(got, ref), (a, len(x))
    finally:
        for h in hs:
            h.free()
