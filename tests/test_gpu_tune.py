"""Launch settings and the autotuner: every setting of every knob must give
the oracle's matches exactly (the knobs move work, they never change what is
found), and the tuner must keep a setting that does the same."""
import itertools

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


def dev(a):
    return torch.from_numpy(np.array(a, np.uint8)).cuda()


def scan_equal(P, h, x, ref):
    n, out = P.pfsm_scan(h, x)
    got = out.cpu().numpy()
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "dfa1024"])
def test_dfa_settings_identical(P, name):
    if name == "cfg1":
        wl = W.cfg1()
    elif name == "cfg2":
        wl = W.cfg2(n=1 << 20)
    else:
        rng = W.rng_for(21)
        d = W.random_table_dfa(rng, 1024, 256, 0.9, 16)
        wl = W.Workload("dfa1024", d, rng.integers(0, 256, 1 << 20, dtype=np.uint8), 21)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    x = dev(wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        occ = P.pfsm_get_option(h, P.PFSM_OPT_MAX_WORKGROUPS_PER_CU)
        assert occ >= 1
        for budget, seg, wpc in itertools.product([-1, 0], [0, 256, 4096, 65536], sorted({0, 1})):
            P.pfsm_set_option(h, P.PFSM_OPT_TABLE_BUDGET, budget)
            P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, seg)
            P.pfsm_set_option(h, P.PFSM_OPT_WORKGROUPS_PER_CU, wpc)
            assert P.pfsm_get_option(h, P.PFSM_OPT_SEGMENT) == seg
            if budget == 0:
                assert P.pfsm_get_option(h, P.PFSM_OPT_RESIDENT_TABLE) == 0
            elif name in ("cfg1", "cfg2"):
                # the default layout keeps tables of up to 256 states in LDS
                assert P.pfsm_get_option(h, P.PFSM_OPT_RESIDENT_TABLE) == 1
            scan_equal(P, h, x, ref)
    finally:
        h.free()


def test_nfa_settings_identical(P):
    wl = W.cfg3(n=1 << 20, n_patterns=200, plant_rate=1e-3)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    x = dev(wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        occ = P.pfsm_get_option(h, P.PFSM_OPT_MAX_WORKGROUPS_PER_CU)
        for pair, seg, wpc in itertools.product([1, 0], [0, 1024, 65536], sorted({0, 1, occ})):
            P.pfsm_set_option(h, P.PFSM_OPT_PAIR_CACHE, pair)
            P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, seg)
            P.pfsm_set_option(h, P.PFSM_OPT_WORKGROUPS_PER_CU, wpc)
            scan_equal(P, h, x, ref)
    finally:
        h.free()


def test_small_segments_grow_lookback(P):
    # 9 MiB in 256-byte segments: more segments than the look-back words a
    # workspace starts with
    wl = W.cfg2(n=9 << 20)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        P.pfsm_set_option(h, P.PFSM_OPT_SEGMENT, 256)
        scan_equal(P, h, dev(wl.data), ref)
    finally:
        h.free()


def test_batch_honours_segment_setting(P):
    rng = np.random.default_rng(31)
    a = W.cfg1().automaton
    b = W.cfg3(n=4096, n_patterns=100).automaton
    lens = rng.integers(1, 30000, 24)
    auts = rng.integers(0, 2, 24).astype(np.int32)
    streams = [rng.choice(list(b"abcd"), n).astype(np.uint8) if t == 0 else
               W.zipf_bytes(rng, int(n)) for n, t in zip(lens, auts)]
    data = np.concatenate(streams)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ha, hb = P.pfsm_load(a), P.pfsm_load(b)
    try:
        P.pfsm_set_option(ha, P.PFSM_OPT_SEGMENT, 512)
        P.pfsm_set_option(hb, P.PFSM_OPT_SEGMENT, 2048)
        n, out, moff = P.pfsm_scan_batch([ha, hb], dev(data), torch.from_numpy(off).cuda(),
                                        torch.from_numpy(auts).cuda())
        out = out.cpu().numpy()
        moff = moff.cpu().numpy()
        for i, (s, t) in enumerate(zip(streams, auts)):
            ref, _ = oracle.scan(a if t == 0 else b, s)
            assert np.array_equal(out[moff[i]:moff[i + 1]], ref), i
    finally:
        ha.free()
        hb.free()


@pytest.mark.parametrize("kind", ["dfa", "nfa"])
def test_tune_keeps_results(P, kind):
    wl = W.cfg2(n=4 << 20) if kind == "dfa" else W.cfg3(n=4 << 20, n_patterns=400, plant_rate=1e-3)
    ref, _ = oracle.scan(wl.automaton, wl.data)
    x = dev(wl.data)
    h = P.pfsm_load(wl.automaton)
    try:
        rep = P.pfsm_tune(h, x, reps=3)
        assert rep["matches"] == len(ref)
        assert rep["configs"] >= 7
        assert 0 < rep["ms_after"] <= rep["ms_before"]
        assert P.pfsm_get_option(h, P.PFSM_OPT_SEGMENT) == rep["segment"]
        assert P.pfsm_get_option(h, P.PFSM_OPT_WORKGROUPS_PER_CU) == rep["workgroups_per_cu"]
        if kind == "dfa":
            assert rep["pair_cache"] == -1 and rep["table_budget"] in (-1, 0)
        else:
            assert rep["table_budget"] == -1 and rep["pair_cache"] in (0, 1)
        scan_equal(P, h, x, ref)
    finally:
        h.free()


def test_option_errors(P):
    hd = P.pfsm_load(W.cfg1().automaton)
    hn = P.pfsm_load(W.fig1_nfa())
    try:
        for bad in (100, 20, 65537, -1):
            with pytest.raises(P.PfsmError) as e:
                P.pfsm_set_option(hd, P.PFSM_OPT_SEGMENT, bad)
            assert e.value.code == P.PFSM_EINVAL
        with pytest.raises(P.PfsmError) as e:
            P.pfsm_set_option(hn, P.PFSM_OPT_TABLE_BUDGET, 0)
        assert e.value.code == P.PFSM_ENOSYS
        with pytest.raises(P.PfsmError) as e:
            P.pfsm_set_option(hd, P.PFSM_OPT_PAIR_CACHE, 0)
        assert e.value.code == P.PFSM_ENOSYS
        with pytest.raises(P.PfsmError) as e:
            P.pfsm_set_option(hd, 99, 0)
        assert e.value.code == P.PFSM_EINVAL
        with pytest.raises(P.PfsmError) as e:
            P.pfsm_set_option(hd, P.PFSM_OPT_MAX_WORKGROUPS_PER_CU, 1)
        assert e.value.code == P.PFSM_EINVAL
    finally:
        hd.free()
        hn.free()
