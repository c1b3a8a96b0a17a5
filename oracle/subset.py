"""Subset construction of an NFA into a DFA (Section II), for tests.

TEST INFRASTRUCTURE ONLY.

Each DFA state is an epsilon-closed set of NFA states; the DFA start is the
closure of {q0}; delta(S, c) is the closure of the union of the targets of
the edges of S whose class holds byte c; the empty set becomes "no
transition" (-1).  A DFA state's label set is the union of the label sets of
its NFA states (a function F -> L generalised to sets, because one DFA state
may stand for finals of several expressions).  The alphabet is the set of
bytes that occur in some class; every other byte maps to -1.
"""
from __future__ import annotations

from typing import Dict, FrozenSet, List, Optional

import numpy as np

from workloads import DFA, label_csr


def _closure(nfa, states) -> FrozenSet[int]:
    out = set(states)
    todo = list(states)
    while todo:
        q = todo.pop()
        for e in range(int(nfa.row_ptr[q]), int(nfa.row_ptr[q + 1])):
            if int(nfa.edge_class[e]) == -1:
                d = int(nfa.edge_dst[e])
                if d not in out:
                    out.add(d)
                    todo.append(d)
    return frozenset(out)


def to_dfa(nfa, max_states: int = 100000, alphabet: Optional[List[int]] = None) -> DFA:
    if alphabet is None:
        alph = set()
        for k in range(nfa.n_classes):
            for b in nfa.class_members(k):
                alph.add(b)
        alphabet = sorted(alph)
    if not alphabet:
        alphabet = [0]
    b2s = -np.ones(256, dtype=np.int16)
    for s, b in enumerate(alphabet):
        b2s[b] = s
    # per-state lists of (byte set, target) for speed
    edges = []
    for q in range(nfa.n_states):
        lst = []
        for e in range(int(nfa.row_ptr[q]), int(nfa.row_ptr[q + 1])):
            k = int(nfa.edge_class[e])
            if k >= 0:
                lst.append((set(nfa.class_members(k)), int(nfa.edge_dst[e])))
        edges.append(lst)
    start = _closure(nfa, [nfa.q0])
    ids: Dict[FrozenSet[int], int] = {start: 0}
    order = [start]
    rows: List[List[int]] = []
    i = 0
    while i < len(order):
        S = order[i]
        row = []
        for b in alphabet:
            tgt = set()
            for q in S:
                for members, d in edges[q]:
                    if b in members:
                        tgt.add(d)
            if not tgt:
                row.append(-1)
                continue
            T = _closure(nfa, tgt)
            if T not in ids:
                if len(order) >= max_states:
                    raise ValueError("subset construction exceeds max_states")
                ids[T] = len(order)
                order.append(T)
            row.append(ids[T])
        rows.append(row)
        i += 1
    finals = {}
    for sid, S in enumerate(order):
        labs = sorted({lab for q in S for lab in nfa.labels_of(q)})
        if labs:
            finals[sid] = labs
    off, lab = label_csr(len(order), finals)
    return DFA(len(order), len(alphabet), 0, b2s, np.asarray(rows, dtype=np.int32).ravel(), off, lab)
