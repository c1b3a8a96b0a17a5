"""The plain definition of the match set, evaluated substring by substring.

TEST INFRASTRUCTURE ONLY (pure Python, tiny inputs).

For every pair 0 <= s <= e < n the automaton is run from scratch on
x[s..e] (Section II semantics: a DFA follows delta; an NFA follows the set of
states reachable through symbol edges with epsilon edges interleaved) and
every label of every final state it ends in is reported as (s, e, label)
(Section III.B reporting rule).  No pruning, no caching, nothing shared
between substrings: O(n^3) set steps.

``work`` counts the scan's work counters (instance-steps T and state
activations X) from their definition, one start at a time.
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


def _coreachable(fsm) -> Set[int]:
    """States from which a final state (non-empty label set) can be reached
    through edges that some byte, or epsilon, can take (reverse search)."""
    n = fsm.n_states
    preds: List[List[int]] = [[] for _ in range(n)]
    if fsm.kind == "dfa":
        used = set(range(fsm.n_symbols)) if fsm.byte_to_symbol is None else \
            {int(v) for v in fsm.byte_to_symbol if int(v) >= 0}
        for q in range(n):
            for s in used:
                t = int(fsm.delta[q * fsm.n_symbols + s])
                if t >= 0:
                    preds[t].append(q)
    else:
        for q in range(n):
            for e in range(int(fsm.row_ptr[q]), int(fsm.row_ptr[q + 1])):
                k = int(fsm.edge_class[e])
                if k == -1 or any(int(w) for w in fsm.class_bits[k * 8:k * 8 + 8]):
                    preds[int(fsm.edge_dst[e])].append(q)
    good = {q for q in range(n) if fsm.labels_of(q)}
    todo = list(good)
    while todo:
        q = todo.pop()
        for p in preds[q]:
            if p not in good:
                good.add(p)
                todo.append(p)
    return good


def work(fsm, x: bytes) -> Tuple[int, int]:
    """The work counters of the scan, from their definition, per start.

    For every start s the instance's state set is advanced one byte at a time
    (epsilon-closed after each byte) and restricted to states that can still
    reach a final state.  T counts the bytes consumed while the set was
    non-empty before the byte (the byte that empties it included); X adds
    the size of the set after each such byte."""
    x = bytes(x)
    good = _coreachable(fsm)
    T = X = 0
    for s in range(len(x)):
        if fsm.kind == "dfa":
            cur: Set[int] = {fsm.q0}
        else:
            cur = _eps_closure(fsm, {fsm.q0})
        for e in range(s, len(x)):
            b = x[e]
            nxt: Set[int] = set()
            if fsm.kind == "dfa":
                sym = b if fsm.byte_to_symbol is None else int(fsm.byte_to_symbol[b])
                if sym >= 0:
                    for q in cur:
                        t = int(fsm.delta[q * fsm.n_symbols + sym])
                        if t >= 0:
                            nxt.add(t)
            else:
                for q in cur:
                    for k in range(int(fsm.row_ptr[q]), int(fsm.row_ptr[q + 1])):
                        c = int(fsm.edge_class[k])
                        if c >= 0 and _in_class(fsm, c, b):
                            nxt.add(int(fsm.edge_dst[k]))
                nxt = _eps_closure(fsm, nxt)
            nxt &= good
            T += 1
            X += len(nxt)
            if not nxt:
                break
            cur = nxt
    return T, X
