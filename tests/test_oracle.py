"""Pins for the CPU oracle: paper examples, closed forms, a library routine
(Python's ``re``), brute force and invariants.  CPU only."""
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import brute, compose, subset, tagset
from workloads.regex import regex_nfa

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def as_set(m):
    return {tuple(int(v) for v in r) for r in np.asarray(m).reshape(-1, 3)}


def as_list(m):
    return [tuple(int(v) for v in r) for r in np.asarray(m).reshape(-1, 3)]


def fig2_golden():
    rows = []
    with open(os.path.join(GOLDEN, "fig2_aacacab.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


# ---------------------------------------------------------------- paper examples

FIG1_REGEXES = [(b"a*c", 0), (b"ac", 1), (b"a(ca)*b", 2)]


@pytest.mark.parametrize("build", ["hand", "regex", "subset_dfa"])
def test_fig2_match_set(build):
    """Fig. 2: exactly the ten printed matches, whatever automaton encodes Fig. 1."""
    fsm = {"hand": W.fig1_nfa, "regex": lambda: regex_nfa(FIG1_REGEXES),
           "subset_dfa": lambda: subset.to_dfa(W.fig1_nfa())}[build]()
    got, _ = oracle.scan(fsm, W.FIG2_INPUT)
    assert as_list(got) == sorted(fig2_golden())


def test_fig2_online_order_of_paper_algorithm():
    """The paper's tagged algorithm reports online in Fig. 2's printing order."""
    assert tagset.run(W.fig1_nfa(), W.FIG2_INPUT) == fig2_golden()


def test_fig3h_three_matches_ending_at_index_1():
    """Fig. 3(h): running Fig. 1's PFSM on "ac" finds three matches ending at 1."""
    got = as_list(oracle.scan(W.fig1_nfa(), b"ac")[0])
    assert len([m for m in got if m[1] == 1]) == 3
    assert got == [(0, 1, 0), (0, 1, 1), (1, 1, 0)]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [0, 1, 2, 7, 64, 300])
def test_sigma_plus_every_substring(n):
    """Sigma+ accepts every non-empty substring: n(n+1)/2 matches, one per (s, e)."""
    rng = np.random.default_rng(n)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    got, work = oracle.scan(W.sigma_plus_dfa(), x)
    assert len(got) == n * (n + 1) // 2
    assert as_set(got) == {(s, e, 0) for s in range(n) for e in range(s, n)}
    # every instance survives to the end of the input: T = X = n(n+1)/2
    assert work["T"] == work["X"] == n * (n + 1) // 2


def test_sigma_plus_bound_with_label_set():
    """|M| <= |L| * n(n+1)/2 (Section III.C), reached with three labels on one state."""
    n = 50
    got, _ = oracle.scan(W.sigma_plus_dfa((4, 1, 9)), bytes(n))
    assert len(got) == 3 * n * (n + 1) // 2
    assert as_list(got)[:3] == [(0, 0, 1), (0, 0, 4), (0, 0, 9)]


@pytest.mark.parametrize("n", [1, 2, 3, 10, 100])
def test_a_plus_on_a_power_n(n):
    fsm = regex_nfa([(b"a+", 3)])
    got, _ = oracle.scan(fsm, b"a" * n)
    assert len(got) == n * (n + 1) // 2


@pytest.mark.parametrize("n", [1, 2, 3, 10, 100])
def test_literal_aa_on_a_power_n(n):
    got, work = oracle.scan(W.literal_dfa(b"aa"), b"a" * n)
    assert as_list(got) == [(s, s + 1, 0) for s in range(n - 1)]
    # each start reads 'a', 'a' (final), then a third symbol that has no
    # transition out of the final state: min(3, n - s) symbols
    assert work["T"] == sum(min(3, n - s) for s in range(n))


def naive_occurrences(hay: bytes, needle: bytes):
    out, i = [], hay.find(needle)
    while i >= 0:
        out.append(i)
        i = hay.find(needle, i + 1)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_literal_equals_overlapping_search(seed):
    """One literal pattern reports exactly the overlapping occurrences bytes.find finds."""
    rng = np.random.default_rng(seed)
    needle = bytes(rng.choice(list(b"ab"), int(rng.integers(1, 5))).astype(np.uint8))
    hay = bytes(rng.choice(list(b"abc"), 3000).astype(np.uint8))
    got = as_list(oracle.scan(W.literal_dfa(needle, 7), hay)[0])
    assert got == [(i, i + len(needle) - 1, 7) for i in naive_occurrences(hay, needle)]


# ---------------------------------------------------------------- library routine: re

REGEXES = [b"a*c", b"ac", b"a(ca)*b", b"(ab|a)*b{1,3}", b"[a-c]+d?", b"a.{0,3}b", b"(a|b)*abb",
           b"[^a]b*", b"(a|ab)(c|bcd)", b"a?a?a?aaa", b"((a|b)(c|d))+", b"d{2,}", b"(a*)*b"]


@pytest.mark.parametrize("pat", REGEXES)
def test_matches_re_fullmatch(pat):
    """Every (s, e) with re.fullmatch(pattern, x[s..e]) and nothing else."""
    rng = np.random.default_rng(len(pat))
    fsm = regex_nfa([(pat, 11)])
    for _ in range(8):
        x = bytes(rng.choice(list(b"abcd"), 40).astype(np.uint8))
        got = as_list(oracle.scan(fsm, x)[0])
        ref = sorted((s, e, 11) for s in range(len(x)) for e in range(s, len(x))
                     if re.fullmatch(pat, x[s:e + 1], re.DOTALL))
        assert got == ref


def test_regex_union_matches_re():
    """A union of expressions (Section III.A) reports each expression's matches with its label."""
    pats = [(REGEXES[i], 100 + i) for i in range(0, len(REGEXES), 2)]
    fsm = regex_nfa(pats)
    rng = np.random.default_rng(5)
    x = bytes(rng.choice(list(b"abcd"), 60).astype(np.uint8))
    got = as_list(oracle.scan(fsm, x)[0])
    ref = sorted((s, e, lab) for s in range(len(x)) for e in range(s, len(x)) for p, lab in pats
                 if re.fullmatch(p, x[s:e + 1], re.DOTALL))
    assert got == ref


# ---------------------------------------------------------------- brute force

def _small_dfa(seed):
    rng = np.random.default_rng(seed)
    return W.random_dfa(rng, int(rng.integers(1, 7)), int(rng.integers(1, 4)), p_dead=0.35,
                        n_finals=int(rng.integers(1, 4)), max_labels=2, n_labels=3), rng


def _small_nfa(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 8))
    return W.random_nfa(rng, n, list(b"abc"), n_edges=int(rng.integers(0, 3 * n + 2)),
                        p_eps=0.25, n_finals=int(rng.integers(1, 4))), rng


@pytest.mark.parametrize("seed", range(40))
def test_dfa_vs_brute_force(seed):
    fsm, rng = _small_dfa(seed)
    x = bytes(rng.choice(list(b"abcd"), int(rng.integers(0, 28))).astype(np.uint8))
    ref = brute.matches(fsm, x)
    for prune in (True, False):
        assert as_list(oracle.scan(fsm, x, prune=prune, threads=3)[0]) == ref


@pytest.mark.parametrize("seed", range(40))
def test_nfa_vs_brute_force(seed):
    fsm, rng = _small_nfa(seed)
    x = bytes(rng.choice(list(b"abcd"), int(rng.integers(0, 28))).astype(np.uint8))
    ref = brute.matches(fsm, x)
    for prune in (True, False):
        for memo in (True, False):
            assert as_list(oracle.scan(fsm, x, prune=prune, memo=memo, threads=2)[0]) == ref


@pytest.mark.parametrize("seed", range(15))
def test_paper_algorithm_vs_brute_force(seed):
    """The tagged four-step algorithm (Section III.B) reaches the plain definition."""
    fsm, rng = _small_nfa(seed)
    x = bytes(rng.choice(list(b"abc"), 20).astype(np.uint8))
    assert sorted(tagset.run(fsm, x)) == brute.matches(fsm, x)


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(12))
def test_nfa_equals_subset_dfa(seed):
    """An NFA and the DFA of its subset construction (Section II) report the same matches."""
    rng = np.random.default_rng(77 + seed)
    fsm = W.random_nfa(rng, 10, list(b"abcd"), n_edges=24, p_eps=0.2, n_finals=3)
    dfa = subset.to_dfa(fsm)
    x = bytes(rng.choice(list(b"abcde"), 3000).astype(np.uint8))
    assert np.array_equal(oracle.scan(fsm, x)[0], oracle.scan(dfa, x)[0])


def test_union_is_union_of_match_sets():
    """Union through an ancillary initial state (Section III.A) reports the union."""
    rng = np.random.default_rng(3)
    parts = [W.random_nfa(rng, 6, list(b"abc"), 14, n_labels=1) for _ in range(3)]
    for i, p in enumerate(parts):  # distinct labels per part
        p.final_labels = p.final_labels * 0 + 10 * i
    parts.append(W.random_dfa(rng, 5, 3, p_dead=0.3, n_labels=1))
    parts[-1].final_labels = parts[-1].final_labels * 0 + 99
    x = bytes(rng.choice(list(b"abcd"), 2000).astype(np.uint8))
    u = compose.union(parts)
    whole = as_set(oracle.scan(u, x)[0])
    assert whole == set().union(*(as_set(oracle.scan(p, x)[0]) for p in parts))


def test_drop_label_equals_filtered():
    """Removing an expression's label removes exactly its matches."""
    wl = W.cfg3(seed=41, n=1 << 16, n_patterns=60, plant_rate=2e-3)
    full, _ = oracle.scan(wl.automaton, wl.data)
    lab = int(full[0, 2])
    a = wl.automaton
    keep = a.final_labels != lab
    off = np.zeros_like(a.final_off)
    for q in range(a.n_states):
        off[q + 1] = off[q] + int(keep[a.final_off[q]:a.final_off[q + 1]].sum())
    b = W.NFA(a.n_states, a.q0, a.n_classes, a.row_ptr, a.edge_class, a.edge_dst, a.class_bits,
              off, a.final_labels[keep])
    assert np.array_equal(oracle.scan(b, wl.data)[0], compose.drop_label(full, lab))


@pytest.mark.parametrize("cuts", [[0, 100, 101, 5000, 8192], [0, 1, 2, 3, 8192], [0, 4096, 8192]])
def test_segment_split_equals_whole(cuts):
    """Lazy data partitioning (Section III.D.2): segments own their starts and read past
    their end; the concatenation equals the whole."""
    wl = W.cfg1(seed=9, n=8192)
    whole, _ = oracle.scan(wl.automaton, wl.data)
    pieces = [oracle.scan(wl.automaton, wl.data, s_lo=a, s_hi=b)[0] for a, b in zip(cuts, cuts[1:])]
    assert np.array_equal(np.concatenate(pieces), whole)


def test_shortcuts_and_threads_do_not_change_results():
    wl = W.cfg3(seed=12, n=1 << 15, n_patterns=80, plant_rate=3e-3)
    ref, _ = oracle.scan(wl.automaton, wl.data, prune=False, memo=False, threads=1)
    assert len(ref) > 10
    for prune in (True, False):
        for memo in (True, False):
            for th in (1, 5):
                got, _ = oracle.scan(wl.automaton, wl.data, prune=prune, memo=memo, threads=th)
                assert np.array_equal(got, ref)


def test_output_sorted_unique_and_in_range():
    wl = W.cfg2(seed=8, n=1 << 18)
    m, work = oracle.scan(wl.automaton, wl.data)
    keys = m[:, 0].astype(np.int64) << 40 | m[:, 1].astype(np.int64) << 8 | m[:, 2]
    assert np.all(np.diff(keys) > 0)
    assert np.all((0 <= m[:, 0]) & (m[:, 0] <= m[:, 1]) & (m[:, 1] < wl.data.size))
    # each planted walk ends in a final state: a match at (plant start, plant end)
    s = as_set(m)
    starts = {(a, a + ln - 1) for a, ln in wl.meta["plants"]}
    assert starts <= {(a, b) for a, b, _ in s}
    assert work["T"] >= wl.data.size


def test_empty_input_and_empty_matches_never_reported():
    # q0 is final (label 5) and has a self loop on 'a': no zero-length matches
    fsm = regex_nfa([(b"a*", 5)])
    assert as_list(oracle.scan(fsm, b"")[0]) == []
    assert as_list(oracle.scan(fsm, b"b")[0]) == []
    assert as_list(oracle.scan(fsm, b"aa")[0]) == [(0, 0, 5), (0, 1, 5), (1, 1, 5)]


def test_invalid_descriptor_rejected():
    d = W.literal_dfa(b"ab")
    d.delta = d.delta.copy()
    d.delta[3] = 99
    with pytest.raises(ValueError):
        oracle.scan(d, b"ab")


def test_log_search_equals_definition():
    # the long-walk workload's search DFA against its plain definition:
    # (s, e) matches when x[s..e] holds no newline and ends with the pattern
    wl = W.log_search(n=1 << 16, line_mean=256)
    x = bytes(wl.data)
    ref, wk = oracle.scan(wl.automaton, x)
    exp = []
    for e in range(4, len(x)):
        if x[e - 4:e + 1] == b"ERROR":
            s = e - 4
            while s >= 0 and x[s] != ord("\n"):
                exp.append((s, e, 0))
                s -= 1
    exp = np.array(sorted(exp), np.int32).reshape(-1, 3)
    assert len(exp) > 100
    assert np.array_equal(ref, exp)
    # every start lives to the end of its line (or of the input)
    nl = [i for i, c in enumerate(x) if c == ord("\n")]
    ends = np.searchsorted(np.array(nl), np.arange(len(x)))
    steps = [(nl[k] if k < len(nl) else len(x) - 1) - s + 1 for s, k in enumerate(ends)]
    assert wk["T"] == sum(steps)


# ---------------------------------------------------------------- generated automata

from hypothesis import given, settings, strategies as st  # noqa: E402


@st.composite
def small_dfas(draw):
    n = draw(st.integers(1, 6))
    s = draw(st.integers(1, 3))
    delta = draw(st.lists(st.integers(-1, n - 1), min_size=n * s, max_size=n * s))
    finals = draw(st.dictionaries(st.integers(0, n - 1), st.lists(st.integers(0, 4), min_size=1, max_size=3),
                                  max_size=n))
    off, lab = W.label_csr(n, finals)
    b2s = -np.ones(256, dtype=np.int16)
    for k in range(s):
        b2s[ord("a") + k] = k
    return W.DFA(n, s, draw(st.integers(0, n - 1)), b2s, np.array(delta, np.int32), off, lab)


@st.composite
def small_nfas(draw):
    n = draw(st.integers(1, 6))
    classes = draw(st.lists(st.sets(st.sampled_from(list(b"abc")), min_size=1, max_size=3), min_size=1, max_size=4))
    edges = draw(st.lists(st.tuples(st.integers(0, n - 1), st.integers(-1, len(classes) - 1), st.integers(0, n - 1)),
                          max_size=3 * n))
    finals = draw(st.dictionaries(st.integers(0, n - 1), st.lists(st.integers(0, 4), min_size=1, max_size=3),
                                  max_size=n))
    src = [e[0] for e in edges]
    cls = [e[1] for e in edges]
    dst = [e[2] for e in edges]
    return W.build_nfa(n, draw(st.integers(0, n - 1)), src, cls, dst, [sorted(c) for c in classes], finals)


@settings(max_examples=150, deadline=None)
@given(small_dfas(), st.binary(max_size=14).map(lambda b: bytes(ord("a") + c % 4 for c in b)))
def test_generated_dfas_vs_brute_force(fsm, x):
    ref = brute.matches(fsm, x)
    for prune in (True, False):
        assert as_list(oracle.scan(fsm, x, prune=prune, threads=2)[0]) == ref


@settings(max_examples=150, deadline=None)
@given(small_nfas(), st.binary(max_size=14).map(lambda b: bytes(ord("a") + c % 4 for c in b)))
def test_generated_nfas_vs_brute_force(fsm, x):
    ref = brute.matches(fsm, x)
    for prune in (True, False):
        for memo in (True, False):
            assert as_list(oracle.scan(fsm, x, prune=prune, memo=memo, threads=2)[0]) == ref


# ---------------------------------------------------------------- work counters of NFAs
#
# T (instance-steps) and X (state activations) are the numerators of the
# reported rates and the GPU's counters are compared with them, so they are
# pinned here by closed forms and by a per-start set simulation.

ANY = list(range(256))


def sigma_plus_union_nfa(k):
    """k copies of Sigma+ under an ancillary initial state (Section III.A):
    q0 -eps-> c_j -any-> f_j -any-> f_j, f_j final with label j."""
    src, cls, dst, finals = [], [], [], {}
    for j in range(k):
        c, f = 1 + 2 * j, 2 + 2 * j
        src += [0, c, f]
        cls += [-1, 0, 0]
        dst += [c, f, f]
        finals[f] = [j]
    return W.build_nfa(1 + 2 * k, 0, src, cls, dst, [ANY], finals)


def literal_chain_nfa(length):
    """q0 -a-> 1 -a-> ... -a-> length (final)."""
    src = list(range(length))
    return W.build_nfa(length + 1, 0, src, [0] * length, [s + 1 for s in src], [[ord("a")]], {length: [0]})


def eps_fanout_nfa(k):
    """q0 -eps-> c_j; c_j -a-> d_j -eps-> e_j -eps-> g_j (g_j final, label j);
    c_j -a-> z_j, from which no final state is reachable."""
    src, cls, dst, finals = [], [], [], {}
    for j in range(k):
        c, d, e, g, z = (1 + 5 * j + i for i in range(5))
        src += [0, c, d, e, c, z]
        cls += [-1, 0, -1, -1, 0, 0]
        dst += [c, d, e, g, z, z]
        finals[g] = [j]
    return W.build_nfa(1 + 5 * k, 0, src, cls, dst, [[ord("a")]], finals)


@pytest.mark.parametrize("k", [1, 2, 5])
@pytest.mark.parametrize("n", [1, 2, 9, 40])
def test_nfa_work_sigma_plus_union(k, n):
    """Every instance lives to the end of the input holding k states: T =
    n(n+1)/2 and X = k n(n+1)/2 (one activation per state per step)."""
    x = np.random.default_rng(n).integers(0, 256, n, dtype=np.uint8)
    for memo in (True, False):
        got, wk = oracle.scan(sigma_plus_union_nfa(k), x, memo=memo, threads=2)
        assert len(got) == k * n * (n + 1) // 2
        assert wk["T"] == n * (n + 1) // 2
        assert wk["X"] == k * n * (n + 1) // 2


@pytest.mark.parametrize("length", [1, 3, 6])
@pytest.mark.parametrize("n", [1, 4, 7, 20])
def test_nfa_work_literal_chain(length, n):
    """a^length on a^n: a start lives min(length, n - s) bytes in one state,
    and the byte after the final state ends it, when there is one."""
    for memo in (True, False):
        got, wk = oracle.scan(literal_chain_nfa(length), b"a" * n, memo=memo, threads=2)
        assert as_list(got) == [(s, s + length - 1, 0) for s in range(n - length + 1)]
        assert wk["T"] == sum(min(length + 1, n - s) for s in range(n))
        assert wk["X"] == sum(min(length, n - s) for s in range(n))


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("n", [1, 2, 10])
def test_nfa_work_epsilon_fan_out(k, n):
    """After one 'a' an instance holds d_j, e_j, g_j for every j (closure
    applied at once; z_j dropped, it reaches no final state): X = 3k per
    start, and the second byte ends it: T = min(2, n - s) per start."""
    for memo in (True, False):
        got, wk = oracle.scan(eps_fanout_nfa(k), b"a" * n, memo=memo, threads=2)
        assert as_list(got) == [(s, s, j) for s in range(n) for j in range(k)]
        assert wk["X"] == 3 * k * n
        assert wk["T"] == sum(min(2, n - s) for s in range(n))


def test_nfa_work_without_pruning_keeps_dead_branch():
    """With pruning off, z_j stays in the set: it is activated once per byte
    the instance reads (first 'a', then every later 'a' on its self loop)."""
    n, k = 6, 2
    _, wk = oracle.scan(eps_fanout_nfa(k), b"a" * n, prune=False, threads=1)
    # per start: 4k states after the first byte (d, e, g, z), then k (z) per byte
    assert wk["X"] == sum(4 * k + k * (n - s - 1) for s in range(n))
    assert wk["T"] == n * (n + 1) // 2


@settings(max_examples=120, deadline=None)
@given(small_nfas(), st.binary(max_size=12).map(lambda b: bytes(ord("a") + c % 4 for c in b)))
def test_generated_nfa_work_vs_per_start_sets(fsm, x):
    T, X = brute.work(fsm, x)
    for memo in (True, False):
        _, wk = oracle.scan(fsm, x, memo=memo, threads=2)
        assert (wk["T"], wk["X"]) == (T, X)


@settings(max_examples=120, deadline=None)
@given(small_dfas(), st.binary(max_size=12).map(lambda b: bytes(ord("a") + c % 4 for c in b)))
def test_generated_dfa_work_vs_per_start_sets(fsm, x):
    assert tuple(oracle.scan(fsm, x, threads=2)[1].values()) == brute.work(fsm, x)


def test_cfg_sample_work_vs_per_start_sets():
    """The NFA union recipe on a short sample: counters equal the per-start
    simulation (chains, byte classes, the any-byte gap states)."""
    wl = W.cfg3(n=600, n_patterns=40, plant_rate=2e-2)
    _, wk = oracle.scan(wl.automaton, wl.data)
    assert (wk["T"], wk["X"]) == brute.work(wl.automaton, bytes(wl.data))
