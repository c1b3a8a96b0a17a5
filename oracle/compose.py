"""Descriptor-level union and label removal, for tests.

TEST INFRASTRUCTURE ONLY.

``union`` puts automata together through a fresh ancillary initial state with
an epsilon edge to each part's initial state (Section III.A); each part keeps
its own final states and labels.  ``drop_label`` is what removing an
expression means for the reported matches: its label is never reported again
(Section III.A: regular expressions can be added or removed).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from workloads import NFA, dfa_as_nfa


def union(parts: Sequence) -> NFA:
    parts = [p if p.kind == "nfa" else dfa_as_nfa(p) for p in parts]
    n = 1 + sum(p.n_states for p in parts)
    src, cls, dst = [], [], []
    bits = []
    finals = {}
    base, cbase = 1, 0
    for p in parts:
        src.append(0); cls.append(-1); dst.append(base + p.q0)
        for q in range(p.n_states):
            for e in range(int(p.row_ptr[q]), int(p.row_ptr[q + 1])):
                k = int(p.edge_class[e])
                src.append(base + q)
                cls.append(k if k < 0 else k + cbase)
                dst.append(base + int(p.edge_dst[e]))
            labs = p.labels_of(q)
            if labs:
                finals[base + q] = labs
        bits.append(np.asarray(p.class_bits, dtype=np.uint32))
        base += p.n_states
        cbase += p.n_classes
    from workloads import build_nfa
    class_bits = np.concatenate(bits) if bits else np.zeros(0, np.uint32)
    return build_nfa(n, 0, src, cls, dst, [], finals, class_bits=class_bits)


def drop_label(matches: np.ndarray, label: int) -> np.ndarray:
    m = np.asarray(matches)
    return m[m[:, 2] != label] if m.size else m
