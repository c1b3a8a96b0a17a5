"""The paper's PFSM algorithm with position tags (Section III.B), in pure Python.

TEST INFRASTRUCTURE ONLY (small inputs).

The active configuration maps each active state to its set of tags, a tag
being the input position at which the instance that reached the state was
started.  For every input position i, in the paper's order:

  1. (re)initialise: q0 becomes active with tag i; states already active stay
     active with their tags;
  2. apply epsilon transitions from the active states until nothing changes,
     each target inheriting the tags of its source;
  3. consume x[i]: select the transitions of the active states whose symbol
     (byte class) contains x[i];
  4. apply them: each target inherits the tags of its source.  The new
     configuration replaces the old one (an instance with no matching
     transition ends).

Reading adopted where the paper is ambiguous: epsilon transitions reached
right after step 4 are applied at once, so that a final state entered by
consuming x[i] and then following epsilon edges is reported with end i.
A match is reported when a final state is entered in step 4 (or its epsilon
closure): (tag, i, label) for every tag and label of that state.  Finals met
in step 2 by the fresh tag would be empty matches and are not reported.

The online order of one step is by start, then label, and steps follow the
input: this is Fig. 2's printing order.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Set, Tuple


def _out_edges(fsm, q: int) -> Iterable[Tuple[int, int]]:
    """(class-or-symbol, target) pairs; class -1 is epsilon.  For a DFA the
    'class' is the symbol index."""
    if fsm.kind == "dfa":
        row = fsm.delta[q * fsm.n_symbols:(q + 1) * fsm.n_symbols]
        return [(s, int(t)) for s, t in enumerate(row) if t >= 0]
    return [(int(fsm.edge_class[e]), int(fsm.edge_dst[e]))
            for e in range(int(fsm.row_ptr[q]), int(fsm.row_ptr[q + 1]))]


def _matches_symbol(fsm, k: int, b: int) -> bool:
    if fsm.kind == "dfa":
        sym = b if fsm.byte_to_symbol is None else int(fsm.byte_to_symbol[b])
        return sym == k
    return k >= 0 and (int(fsm.class_bits[k * 8 + (b >> 5)]) >> (b & 31)) & 1 == 1


def _apply_epsilon(fsm, active: Dict[int, Set[int]]) -> None:
    changed = True
    while changed:
        changed = False
        for q in list(active):
            for k, d in _out_edges(fsm, q):
                if fsm.kind == "nfa" and k == -1:
                    tags = active.setdefault(d, set())
                    before = len(tags)
                    tags |= active[q]
                    if len(tags) != before:
                        changed = True


def run(fsm, x: bytes) -> List[Tuple[int, int, int]]:
    """All matches as (start, end, label) in the PFSM's online order."""
    active: Dict[int, Set[int]] = {}
    out: List[Tuple[int, int, int]] = []
    for i, b in enumerate(bytes(x)):
        # step 1: reinitialisation with tag i; active states are kept
        active.setdefault(fsm.q0, set()).add(i)
        # step 2: epsilon transitions, tags propagated
        _apply_epsilon(fsm, active)
        # steps 3 and 4: transitions matching x[i], tags propagated
        nxt: Dict[int, Set[int]] = {}
        for q, tags in active.items():
            for k, d in _out_edges(fsm, q):
                if _matches_symbol(fsm, k, b):
                    nxt.setdefault(d, set()).update(tags)
        _apply_epsilon(fsm, nxt)
        # report every final state entered in this step
        step = set()
        for q, tags in nxt.items():
            for lab in fsm.labels_of(q):
                for t in tags:
                    step.add((t, lab))
        out.extend((t, i, lab) for t, lab in sorted(step))
        active = nxt
    return out
