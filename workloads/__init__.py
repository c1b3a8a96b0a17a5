"""Seeded synthetic workloads for the all-matches PFSM scan.

This package only *builds* inputs: automaton descriptors (the PFSM tuple of
Section III.A, with the union through an ancillary initial state) and input
byte streams.  It computes no matches and holds none of the scan's
arithmetic, so both the CPU oracle and the GPU library can consume what it
produces without sharing any matching code.

Descriptor layout (mirrors the C-ABI structs ``pfsm_dfa_desc`` and
``pfsm_nfa_desc``):

* ``DFA``: dense row-major transition table ``delta[n_states * n_symbols]``
  (target state or -1 = no transition), an optional ``byte_to_symbol[256]``
  map (-1 = byte outside the alphabet; ``None`` = identity, 256 symbols) and
  the per-state label set as CSR (``final_off``, ``final_labels``).
* ``NFA``: CSR successor lists (``row_ptr``, ``edge_class``, ``edge_dst``);
  class -1 is an epsilon edge, class k >= 0 is the 256-bit byte set stored in
  ``class_bits[k*8:(k+1)*8]`` (bit b%32 of word b//32 set when byte b is in
  the class); label CSR as for the DFA.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

MiB = 1 << 20
KiB = 1 << 10


def rng_for(seed: int) -> np.random.Generator:
    """The one PRNG every workload draws from: numpy PCG64 with the given seed."""
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Descriptors
# --------------------------------------------------------------------------


@dataclass
class DFA:
    n_states: int
    n_symbols: int
    q0: int
    byte_to_symbol: Optional[np.ndarray]  # int16[256] or None (identity)
    delta: np.ndarray  # int32[n_states * n_symbols]
    final_off: np.ndarray  # int32[n_states + 1]
    final_labels: np.ndarray  # int32[nnz]
    kind: str = field(default="dfa", init=False)

    def labels_of(self, q: int) -> List[int]:
        return [int(v) for v in self.final_labels[self.final_off[q]:self.final_off[q + 1]]]


@dataclass
class NFA:
    n_states: int
    q0: int
    n_classes: int
    row_ptr: np.ndarray  # int32[n_states + 1]
    edge_class: np.ndarray  # int32[n_edges], -1 = epsilon
    edge_dst: np.ndarray  # int32[n_edges]
    class_bits: np.ndarray  # uint32[n_classes * 8]
    final_off: np.ndarray  # int32[n_states + 1]
    final_labels: np.ndarray  # int32[nnz]
    kind: str = field(default="nfa", init=False)

    @property
    def n_edges(self) -> int:
        return int(self.row_ptr[-1])

    def labels_of(self, q: int) -> List[int]:
        return [int(v) for v in self.final_labels[self.final_off[q]:self.final_off[q + 1]]]

    def class_members(self, k: int) -> List[int]:
        words = self.class_bits[k * 8:(k + 1) * 8]
        return [b for b in range(256) if (int(words[b >> 5]) >> (b & 31)) & 1]


def label_csr(n_states: int, finals: Dict[int, Iterable[int]]) -> Tuple[np.ndarray, np.ndarray]:
    """CSR of per-state label lists, in the order given."""
    off = np.zeros(n_states + 1, dtype=np.int32)
    lab: List[int] = []
    for q in range(n_states):
        ls = list(finals.get(q, ()))
        lab.extend(ls)
        off[q + 1] = off[q] + len(ls)
    return off, np.asarray(lab, dtype=np.int32)


def class_bits_of(classes: Sequence[Iterable[int]]) -> np.ndarray:
    bits = np.zeros(len(classes) * 8, dtype=np.uint32)
    for k, members in enumerate(classes):
        for b in members:
            bits[k * 8 + (b >> 5)] |= np.uint32(1 << (b & 31))
    return bits


def build_nfa(n_states: int, q0: int, src, cls, dst, classes: Sequence[Iterable[int]],
              finals: Dict[int, Iterable[int]], class_bits: Optional[np.ndarray] = None) -> NFA:
    """Pack an edge list (src, class, dst) into the CSR descriptor.

    Edges keep their relative order within a source state (stable sort).
    """
    src = np.asarray(src, dtype=np.int64)
    cls = np.asarray(cls, dtype=np.int32)
    dst = np.asarray(dst, dtype=np.int32)
    order = np.argsort(src, kind="stable")
    counts = np.bincount(src, minlength=n_states) if src.size else np.zeros(n_states, np.int64)
    row_ptr = np.zeros(n_states + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(counts)
    off, lab = label_csr(n_states, finals)
    if class_bits is None:
        class_bits = class_bits_of(classes)
    return NFA(n_states=n_states, q0=q0, n_classes=len(class_bits) // 8,
               row_ptr=row_ptr, edge_class=cls[order].copy(), edge_dst=dst[order].copy(),
               class_bits=class_bits, final_off=off, final_labels=lab)


def dfa_as_nfa(d: DFA) -> NFA:
    """The same automaton with its dense table written as CSR successor lists.

    One class per symbol: the set of bytes that map to it.
    """
    if d.byte_to_symbol is None:
        sym_bytes = [[s] for s in range(d.n_symbols)]
    else:
        sym_bytes = [[] for _ in range(d.n_symbols)]
        for b in range(256):
            s = int(d.byte_to_symbol[b])
            if s >= 0:
                sym_bytes[s].append(b)
    tbl = d.delta.reshape(d.n_states, d.n_symbols)
    qs, ss = np.nonzero(tbl >= 0)
    finals = {q: d.labels_of(q) for q in range(d.n_states) if d.final_off[q + 1] > d.final_off[q]}
    return build_nfa(d.n_states, d.q0, qs, ss, tbl[qs, ss], sym_bytes, finals)


# --------------------------------------------------------------------------
# Fixtures
# --------------------------------------------------------------------------


def fig1_nfa() -> NFA:
    """A PFSM for the three expressions of Fig. 1 (the figure's image is lost).

    Labels follow the order in which Section III.A names the expressions:
    0 = "a*c", 1 = "ac", 2 = "a(ca)*b".  The ancillary initial state 0 has
    epsilon edges to each component's start (Section III.A union).
    Byte classes: 0 = {'a'}, 1 = {'b'}, 2 = {'c'}.
    """
    a, b, c = 0, 1, 2
    # states: 0 = q0; "a*c": 1 -> 2; "ac": 3 -> 4 -> 5; "a(ca)*b": 6 -> 7 <-> 8, 7 -> 9
    edges = [
        (0, -1, 1), (0, -1, 3), (0, -1, 6),
        (1, a, 1), (1, c, 2),
        (3, a, 4), (4, c, 5),
        (6, a, 7), (7, c, 8), (8, a, 7), (7, b, 9),
    ]
    src, cls, dst = zip(*edges)
    return build_nfa(10, 0, src, cls, dst, [[ord("a")], [ord("b")], [ord("c")]],
                     {2: [0], 5: [1], 9: [2]})


FIG2_INPUT = b"aacacab"


def sigma_plus_dfa(labels: Sequence[int] = (0,)) -> DFA:
    """Sigma+ over all bytes: every non-empty substring matches (closed form n(n+1)/2)."""
    delta = np.ones(2 * 256, dtype=np.int32)
    off, lab = label_csr(2, {1: list(labels)})
    return DFA(2, 256, 0, None, delta, off, lab)


def literal_dfa(pattern: bytes, label: int = 0) -> DFA:
    """Exact-literal DFA (no failure links): state k = k bytes of the pattern read."""
    m = len(pattern)
    delta = -np.ones((m + 1) * 256, dtype=np.int32)
    for k, ch in enumerate(pattern):
        delta[k * 256 + ch] = k + 1
    off, lab = label_csr(m + 1, {m: [label]})
    return DFA(m + 1, 256, 0, None, delta, off, lab)


def kmp_dfa(pattern: bytes, kill: bytes = b"\n", label: int = 0) -> DFA:
    """Search DFA for ``[^kill]*pattern`` over bytes (the Knuth-Morris-Pratt
    automaton: state q = the longest prefix of the pattern that ends here);
    a kill byte has no transition, so an instance lives until the next one."""
    m = len(pattern)
    delta = np.zeros((m + 1, 256), dtype=np.int32)
    delta[0, pattern[0]] = 1
    back = 0
    for q in range(1, m + 1):
        delta[q] = delta[back]
        if q < m:
            delta[q, pattern[q]] = q + 1
            back = int(delta[back, pattern[q]])
    for k in kill:
        delta[:, k] = -1
    off, lab = label_csr(m + 1, {m: [label]})
    return DFA(m + 1, 256, 0, None, delta.ravel(), off, lab)


# --------------------------------------------------------------------------
# Random small automata for property tests
# --------------------------------------------------------------------------


def random_dfa(rng: np.random.Generator, n_states: int, n_symbols: int, p_dead: float = 0.5,
               n_finals: int = 2, max_labels: int = 2, n_labels: int = 4,
               alphabet: Optional[Sequence[int]] = None) -> DFA:
    """Small random DFA; finals carry 1..max_labels labels drawn from 0..n_labels-1."""
    tbl = rng.integers(0, n_states, (n_states, n_symbols))
    tbl[rng.random((n_states, n_symbols)) < p_dead] = -1
    finals = {}
    for q in rng.choice(n_states, min(n_finals, n_states), replace=False):
        k = int(rng.integers(1, min(max_labels, n_labels) + 1))
        finals[int(q)] = [int(v) for v in rng.choice(n_labels, k, replace=False)]
    off, lab = label_csr(n_states, finals)
    b2s = None
    if alphabet is not None or n_symbols != 256:
        if alphabet is None:
            alphabet = list(range(ord("a"), ord("a") + n_symbols))
        b2s = -np.ones(256, dtype=np.int16)
        for s, bt in enumerate(alphabet):
            b2s[bt] = s
    return DFA(n_states, n_symbols, int(rng.integers(0, n_states)), b2s,
               tbl.astype(np.int32).ravel(), off, lab)


def random_nfa(rng: np.random.Generator, n_states: int, alphabet: Sequence[int], n_edges: int,
               p_eps: float = 0.15, max_class: int = 3, n_finals: int = 3, max_labels: int = 2,
               n_labels: int = 4) -> NFA:
    """Small random NFA with epsilon edges, byte classes, cycles and label sets."""
    classes: List[List[int]] = []
    src, cls, dst = [], [], []
    for _ in range(n_edges):
        s, d = int(rng.integers(0, n_states)), int(rng.integers(0, n_states))
        if rng.random() < p_eps:
            c = -1
        else:
            k = int(rng.integers(1, max_class + 1))
            classes.append([int(v) for v in rng.choice(alphabet, min(k, len(alphabet)), replace=False)])
            c = len(classes) - 1
        src.append(s); cls.append(c); dst.append(d)
    finals = {}
    for q in rng.choice(n_states, min(n_finals, n_states), replace=False):
        k = int(rng.integers(1, min(max_labels, n_labels) + 1))
        finals[int(q)] = [int(v) for v in rng.choice(n_labels, k, replace=False)]
    return build_nfa(n_states, int(rng.integers(0, n_states)), src, cls, dst, classes, finals)


# --------------------------------------------------------------------------
# Benchmark configurations
# --------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    automaton: object  # DFA or NFA
    data: np.ndarray  # uint8 input
    seed: int
    meta: dict = field(default_factory=dict)


def _plant_walk(rng: np.random.Generator, d: DFA, live: List[np.ndarray], sym_byte: np.ndarray,
                cap: int = 64) -> np.ndarray:
    """Random walk over defined transitions from q0 until the first final state.

    Restarts on a dead end or when the walk reaches ``cap`` bytes.
    """
    tbl = d.delta.reshape(d.n_states, d.n_symbols)
    is_final = np.diff(d.final_off) > 0
    while True:
        q, out = d.q0, []
        while len(out) < cap:
            opts = live[q]
            if opts.size == 0:
                break
            s = int(opts[rng.integers(0, opts.size)])
            q = int(tbl[q, s])
            out.append(int(sym_byte[s]))
            if is_final[q]:
                return np.asarray(out, dtype=np.uint8)
        # dead end or cap reached: draw a fresh walk


def random_table_dfa(rng: np.random.Generator, n_states: int, n_symbols: int, p_dead: float,
                     n_finals: int, final_lo: int = 1) -> DFA:
    """Dense random DFA: each entry is -1 with probability p_dead, else uniform."""
    dead = rng.random((n_states, n_symbols)) < p_dead
    tgt = rng.integers(0, n_states, (n_states, n_symbols))
    delta = np.where(dead, -1, tgt).astype(np.int32).ravel()
    fin = rng.choice(np.arange(final_lo, n_states), n_finals, replace=False)
    off, lab = label_csr(n_states, {int(q): [k] for k, q in enumerate(fin)})
    return DFA(n_states, n_symbols, 0, None, delta, off, lab)


def cfg1(seed: int = 1, n: int = 4096) -> Workload:
    """16-state random DFA over {a,b,c,d} (dead sink p=0.6), 4 KiB uniform input."""
    rng = rng_for(seed)
    d = random_table_dfa(rng, 16, 4, 0.6, 2)
    b2s = -np.ones(256, dtype=np.int16)
    b2s[ord("a"):ord("a") + 4] = np.arange(4)
    d.byte_to_symbol = b2s
    x = (rng.integers(0, 4, n) + ord("a")).astype(np.uint8)
    return Workload("random DFA 16 states x 4 symbols, 4 KiB abcd input", d, x, seed)


def cfg2(seed: int = 2, n: int = 16 * MiB, plant_every: int = 4 * KiB) -> Workload:
    """256-state random DFA over bytes (dead p=0.9, 16 finals), 16 MiB uniform bytes
    with one accepting walk planted per 4 KiB block."""
    rng = rng_for(seed)
    d = random_table_dfa(rng, 256, 256, 0.9, 16)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    tbl = d.delta.reshape(d.n_states, d.n_symbols)
    live = [np.nonzero(tbl[q] >= 0)[0] for q in range(d.n_states)]
    sym_byte = np.arange(256)
    plants = []
    for blk in range(n // plant_every):
        w = _plant_walk(rng, d, live, sym_byte)
        off = blk * plant_every + int(rng.integers(0, plant_every - w.size + 1))
        x[off:off + w.size] = w
        plants.append((off, w.size))
    size = f"{n >> 20} MiB" if n % MiB == 0 else f"{n} B"
    return Workload(f"random DFA 256 states x 256 symbols, {size} uniform bytes + planted walks",
                    d, x, seed, {"plants": plants})


def zipf_bytes(rng: np.random.Generator, n: int, s: float = 1.1, perm: Optional[np.ndarray] = None,
               chunk: int = 8 * MiB) -> np.ndarray:
    """i.i.d. bytes with P(rank k) proportional to k^-s over 256 ranks; rank->byte by ``perm``."""
    k = np.arange(1, 257, dtype=np.float64)
    p = k ** -s
    cdf = np.cumsum(p / p.sum())
    cdf[-1] = 1.0
    if perm is None:
        perm = rng.permutation(256).astype(np.uint8)
    out = np.empty(n, dtype=np.uint8)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = perm[np.searchsorted(cdf, rng.random(hi - lo), side="right")]
    return out


@dataclass
class Signature:
    edge_sets: List[List[int]]  # byte set of each chain edge, in order
    gap_before: int  # index of the edge preceded by a .{0,gap_max} gap, or -1
    label: int


def signature_union(rng: np.random.Generator, n_patterns: int = 2000, len_lo: int = 6,
                    len_hi: int = 40, p_class: float = 0.2, class_lo: int = 2, class_hi: int = 16,
                    frac_gap: float = 0.05, gap_max: int = 64, label_base: int = 0):
    """Signature patterns: chains of len_lo..len_hi states; each edge one byte (1-p_class)
    or a class of class_lo..class_hi distinct bytes; a fraction carry one .{0,gap_max} gap
    at an interior edge.  Returns the pattern list (pure data)."""
    pats = []
    gap_set = set(int(v) for v in rng.choice(n_patterns, int(round(frac_gap * n_patterns)),
                                             replace=False)) if frac_gap > 0 else set()
    for p in range(n_patterns):
        n_states = int(rng.integers(len_lo, len_hi + 1))
        sets = []
        for _ in range(n_states - 1):
            if rng.random() < p_class:
                k = int(rng.integers(class_lo, class_hi + 1))
                sets.append(sorted(int(v) for v in rng.choice(256, k, replace=False)))
            else:
                sets.append([int(rng.integers(0, 256))])
        gap = int(rng.integers(1, n_states - 1)) if p in gap_set else -1
        pats.append(Signature(sets, gap, label_base + p))
    return pats


def signature_component(sig: Signature, first_state: int, gap_max: int = 64):
    """Edges of one signature as a chain component whose states start at ``first_state``.

    A gap before edge j is 64 any-byte states g_1..g_64 after chain state c_j:
    c_j -any-> g_1 -any-> ... -any-> g_64, and each g_k also carries edge j.
    Returns (n_states, edges[(src, class_key, dst)], final_state); class keys are
    ('b', byte), ('any',) or ('set', tuple).
    """
    m = len(sig.edge_sets) + 1
    edges = []

    def key(sset):
        return ("b", sset[0]) if len(sset) == 1 else ("set", tuple(sset))

    for j, sset in enumerate(sig.edge_sets):
        edges.append((first_state + j, key(sset), first_state + j + 1))
    n = m
    if sig.gap_before >= 0:
        j = sig.gap_before
        g0 = first_state + m
        post = key(sig.edge_sets[j])
        edges.append((first_state + j, ("any",), g0))
        for k in range(gap_max):
            if k + 1 < gap_max:
                edges.append((g0 + k, ("any",), g0 + k + 1))
            edges.append((g0 + k, post, first_state + j + 1))
        n += gap_max
    return n, edges, first_state + m - 1


def union_nfa(sigs: Sequence[Signature], gap_max: int = 64) -> NFA:
    """Union of signature chains under an ancillary initial state 0 (Section III.A)."""
    edges_all = []
    finals = {}
    nxt = 1
    for sig in sigs:
        n, edges, fin = signature_component(sig, nxt, gap_max)
        edges_all.append((0, ("eps",), nxt))
        edges_all.extend(edges)
        finals[fin] = [sig.label]
        nxt += n
    # class numbering: 0..255 singletons, 256 = any byte, then multi-byte sets in order
    set_ids: Dict[tuple, int] = {}
    classes: List[List[int]] = [[b] for b in range(256)] + [list(range(256))]
    src = np.empty(len(edges_all), np.int64)
    cls = np.empty(len(edges_all), np.int32)
    dst = np.empty(len(edges_all), np.int32)
    for i, (s, k, d) in enumerate(edges_all):
        if k[0] == "eps":
            c = -1
        elif k[0] == "b":
            c = k[1]
        elif k[0] == "any":
            c = 256
        else:
            c = set_ids.get(k[1])
            if c is None:
                c = len(classes)
                set_ids[k[1]] = c
                classes.append(list(k[1]))
        src[i], cls[i], dst[i] = s, c, d
    return build_nfa(nxt, 0, src, cls, dst, classes, finals)


def _instance_bytes(rng: np.random.Generator, sig: Signature, gap_max: int, perm: np.ndarray) -> np.ndarray:
    out = []
    for j, sset in enumerate(sig.edge_sets):
        if j == sig.gap_before:
            g = int(rng.integers(0, gap_max + 1))
            if g:
                out.extend(int(v) for v in zipf_bytes(rng, g, perm=perm))
        out.append(sset[int(rng.integers(0, len(sset)))])
    return np.asarray(out, dtype=np.uint8)


def cfg3(seed: int = 3, n: int = 64 * MiB, n_patterns: int = 2000, plant_rate: float = 1e-4) -> Workload:
    """NFA union of 2,000 signature chains (~52k states, CSR), 64 MiB Zipf(1.1) input
    with pattern instances planted at plant_rate per byte, never overlapping."""
    rng = rng_for(seed)
    sigs = signature_union(rng, n_patterns)
    nfa = union_nfa(sigs)
    perm = rng.permutation(256).astype(np.uint8)
    x = zipf_bytes(rng, n, perm=perm)
    n_plants = int(round(n * plant_rate))
    plants = []
    if n_plants:
        blk = n // n_plants
        for i in range(n_plants):
            sig = sigs[int(rng.integers(0, len(sigs)))]
            w = _instance_bytes(rng, sig, 64, perm)
            if w.size > blk:
                continue
            off = i * blk + int(rng.integers(0, blk - w.size + 1))
            x[off:off + w.size] = w
            plants.append((off, w.size, sig.label))
    return Workload(f"NFA union of {n_patterns} signature chains, {n >> 20} MiB Zipf(1.1) bytes",
                    nfa, x, seed, {"plants": plants, "signatures": sigs, "perm": perm})


def log_search(seed: int = 6, n: int = 16 * MiB, line_mean: int = 1024, pattern: bytes = b"ERROR",
               hits_per_line: float = 0.5) -> Workload:
    """Long walks: the ``[^\n]*ERROR`` search DFA over text lines.  Bytes are
    lowercase letters and spaces, each byte a newline with probability
    1/line_mean; the pattern is written at uniform positions, about
    hits_per_line times per line.  Every start stays live until the end of
    its line, so a per-start walk averages about line_mean/2 steps."""
    rng = rng_for(seed)
    alpha = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz ", np.uint8)
    x = alpha[rng.integers(0, alpha.size, n)]
    x[rng.random(n) < 1.0 / line_mean] = ord("\n")
    k = int(n / line_mean * hits_per_line)
    pat = np.frombuffer(pattern, np.uint8)
    for off in rng.integers(0, max(1, n - pat.size), k):
        x[off:off + pat.size] = pat
    return Workload(f"log search [^\\n]*{pattern.decode()}, lines ~{line_mean} B, {n} B", kmp_dfa(pattern), x, seed,
                    {"line_mean": line_mean})


@dataclass
class BatchWorkload:
    name: str
    automata: list  # DFAs and NFAs, indexed by stream_automaton
    data: np.ndarray  # every stream, concatenated (uint8)
    stream_off: np.ndarray  # int64 [n_streams + 1]
    stream_automaton: np.ndarray  # int32 [n_streams]
    seed: int
    ops: list = field(default_factory=list)  # edits of the NFA between batches
    meta: dict = field(default_factory=dict)


def _plant_pool_dfa(rng: np.random.Generator, d: DFA, k: int) -> List[np.ndarray]:
    tbl = d.delta.reshape(d.n_states, d.n_symbols)
    live = [np.nonzero(tbl[q] >= 0)[0] for q in range(d.n_states)]
    return [_plant_walk(rng, d, live, np.arange(256)) for _ in range(k)]


def cfg4(seed: int = 4, n_streams: int = 4096, len_lo: int = 64, len_hi: int = MiB,
         dfa_states: Sequence[int] = (256, 1024, 2048, 4096), n_patterns: int = 2000, n_ops: int = 100,
         plant_every: int = 4 * KiB, plant_rate: float = 1e-4, pool: int = 256) -> BatchWorkload:
    """Batched scan: four random byte DFAs of 256-4,096 states (cfg2 recipe:
    dead entries p=0.9, 16 finals) and one NFA union of signature chains (cfg3
    recipe); n_streams streams with lengths log-uniform on [len_lo, len_hi],
    each assigned a uniformly drawn automaton.  DFA streams hold uniform bytes
    with one accepting walk planted per 4 KiB; NFA streams hold Zipf(1.1)
    bytes with signature instances planted at plant_rate per byte.  Planted
    strings are drawn from a seeded pool of `pool` per automaton.  ``ops``
    lists n_ops edits of the NFA, alternately adding a fresh chain with a new
    label and removing a uniformly drawn present label."""
    rng = rng_for(seed)
    dfas = [random_table_dfa(rng, int(n), 256, 0.9, 16) for n in dfa_states]
    sigs = signature_union(rng, n_patterns)
    nfa = union_nfa(sigs)
    perm = rng.permutation(256).astype(np.uint8)
    automata = list(dfas) + [nfa]
    nfa_idx = len(dfas)
    lens = np.exp(rng.uniform(np.log(len_lo), np.log(len_hi), n_streams)).astype(np.int64)
    aut = rng.integers(0, len(automata), n_streams).astype(np.int32)
    off = np.zeros(n_streams + 1, np.int64)
    off[1:] = np.cumsum(lens)
    data = rng.integers(0, 256, int(off[-1]), dtype=np.uint8)
    pools = [_plant_pool_dfa(rng, d, pool) for d in dfas]
    inst = [_instance_bytes(rng, sigs[int(rng.integers(0, len(sigs)))], 64, perm) for _ in range(pool)]
    for s in range(n_streams):
        lo, hi = int(off[s]), int(off[s + 1])
        n = hi - lo
        if aut[s] == nfa_idx:
            data[lo:hi] = zipf_bytes(rng, n, perm=perm)
            for _ in range(int(rng.binomial(n, plant_rate))):
                w = inst[int(rng.integers(0, pool))]
                if w.size <= n:
                    at = lo + int(rng.integers(0, n - w.size + 1))
                    data[at:at + w.size] = w
        else:
            pl = pools[int(aut[s])]
            for blk in range(n // plant_every):
                w = pl[int(rng.integers(0, pool))]
                at = lo + blk * plant_every + int(rng.integers(0, plant_every - w.size + 1))
                data[at:at + w.size] = w
    ops = []
    present = [s.label for s in sigs]
    nxt = n_patterns
    for i in range(n_ops):
        if i % 2 == 0:
            sig = signature_union(rng, 1, label_base=nxt)
            ops.append(("add", union_nfa(sig), [nxt]))
            present.append(nxt)
            nxt += 1
        else:
            lab = present.pop(int(rng.integers(0, len(present))))
            ops.append(("remove", lab))
    return BatchWorkload(f"{n_streams} streams log-uniform {len_lo} B-{len_hi >> 10} KiB over 4 random DFAs "
                         f"({'/'.join(str(int(n)) for n in dfa_states)} states) and an NFA union of "
                         f"{n_patterns} signatures", automata, data, off, aut, seed, ops,
                         {"nfa_index": nfa_idx, "signatures": sigs, "perm": perm})


@dataclass
class ServeWorkload:
    name: str
    automata: list  # 4 small byte-mapped DFAs, then 4 NFA unions
    pools: list  # per automaton: request payload buffers to slice from
    seed: int
    len_lo: int
    len_hi: int
    meta: dict = field(default_factory=dict)

    def requests(self, rng: np.random.Generator, n: int):
        """n requests: (automaton, bytes) with a uniformly drawn automaton and a
        length log-uniform on [len_lo, len_hi], cut from that automaton's pool."""
        out = []
        for _ in range(n):
            a = int(rng.integers(0, len(self.automata)))
            k = int(np.exp(rng.uniform(np.log(self.len_lo), np.log(self.len_hi))))
            buf = self.pools[a][int(rng.integers(0, len(self.pools[a])))]
            at = int(rng.integers(0, buf.size - k + 1))
            out.append((a, buf[at:at + k]))
        return out


def cfg5(seed: int = 5, len_lo: int = 256, len_hi: int = 4 * MiB, n_patterns: int = 2000,
         pool_per_automaton: int = 4) -> ServeWorkload:
    """Served scans: 8 resident automata (the cfg1 recipe with seeds 5-8, the
    cfg3 NFA recipe with seeds 9-12); requests log-uniform on [256 B, 4 MiB]
    (mean about 432 KB), bytes over 'abcd' for the DFAs and Zipf(1.1) bytes
    for the NFAs (each NFA's own byte permutation, instances planted at 1e-4
    per byte).  Payloads are slices of per-automaton pools of len_hi bytes."""
    automata, pools = [], []
    for sd in range(seed, seed + 4):
        automata.append(cfg1(seed=sd).automaton)
        rng = rng_for(1000 + sd)
        pools.append([(rng.integers(0, 4, len_hi) + ord("a")).astype(np.uint8) for _ in range(pool_per_automaton)])
    for sd in range(seed + 4, seed + 8):
        rng = rng_for(sd)
        sigs = signature_union(rng, n_patterns)
        automata.append(union_nfa(sigs))
        perm = rng.permutation(256).astype(np.uint8)
        bufs = []
        for _ in range(pool_per_automaton):
            x = zipf_bytes(rng, len_hi, perm=perm)
            for _ in range(int(len_hi * 1e-4)):
                w = _instance_bytes(rng, sigs[int(rng.integers(0, len(sigs)))], 64, perm)
                at = int(rng.integers(0, len_hi - w.size + 1))
                x[at:at + w.size] = w
            bufs.append(x)
        pools.append(bufs)
    return ServeWorkload("8 resident automata (4 random DFAs of 16 states over abcd, 4 NFA unions of "
                         f"{n_patterns} signatures); requests log-uniform {len_lo} B-{len_hi >> 20} MiB",
                         automata, pools, seed, len_lo, len_hi)
