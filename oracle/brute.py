"""The plain definition of the match set, evaluated substring by substring.

TEST INFRASTRUCTURE ONLY (pure Python, tiny inputs).

For every pair 0 <= s <= e < n the automaton is run from scratch on
x[s..e] (Section II semantics: a DFA follows delta; an NFA follows the set of
states reachable through symbol edges with epsilon edges interleaved) and
every label of every final state it ends in is reported as (s, e, label)
(Section III.B reporting rule).  No pruning, no caching, nothing shared
between substrings: O(n^3) set steps.
"""
from __future__ import annotations

from typing import List, Set, Tuple


def _dfa_accepting_labels(d, sub: bytes) -> Set[int]:
    q = d.q0
    for b in sub:
        sym = b if d.byte_to_symbol is None else int(d.byte_to_symbol[b])
        if sym < 0:
            return set()
        q = int(d.delta[q * d.n_symbols + sym])
        if q < 0:
            return set()
    return set(d.labels_of(q))


def _eps_closure(a, states: Set[int]) -> Set[int]:
    out = set(states)
    todo = list(states)
    while todo:
        q = todo.pop()
        for e in range(int(a.row_ptr[q]), int(a.row_ptr[q + 1])):
            if int(a.edge_class[e]) == -1:
                d = int(a.edge_dst[e])
                if d not in out:
                    out.add(d)
                    todo.append(d)
    return out


def _in_class(a, k: int, b: int) -> bool:
    return (int(a.class_bits[k * 8 + (b >> 5)]) >> (b & 31)) & 1 == 1


def _nfa_accepting_labels(a, sub: bytes) -> Set[int]:
    cur = _eps_closure(a, {a.q0})
    for b in sub:
        nxt = set()
        for q in cur:
            for e in range(int(a.row_ptr[q]), int(a.row_ptr[q + 1])):
                k = int(a.edge_class[e])
                if k >= 0 and _in_class(a, k, b):
                    nxt.add(int(a.edge_dst[e]))
        cur = _eps_closure(a, nxt)
        if not cur:
            return set()
    labs: Set[int] = set()
    for q in cur:
        labs.update(a.labels_of(q))
    return labs


def matches(fsm, x: bytes) -> List[Tuple[int, int, int]]:
    """Sorted list of (start, end, label), end inclusive, over all substrings."""
    x = bytes(x)
    run = _dfa_accepting_labels if fsm.kind == "dfa" else _nfa_accepting_labels
    out = []
    for s in range(len(x)):
        for e in range(s, len(x)):
            for lab in run(fsm, x[s:e + 1]):
                out.append((s, e, lab))
    return sorted(out)
