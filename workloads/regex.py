"""Regular expressions to epsilon-NFA descriptors (Thompson construction).

Builds test automata from small regular expressions over bytes; it computes
no matches.  Supported syntax: literal bytes, ``.`` (any byte), ``[...]``
classes with ranges and leading ``^``, ``\\`` escapes, grouping ``( )``,
alternation ``|``, and the postfix operators ``*``, ``+``, ``?``, ``{m}``,
``{m,}``, ``{m,n}``.  Several expressions are put together through an
ancillary initial state with an epsilon edge to each expression's start
(Section III.A); the final state of expression i carries its label.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

from workloads import NFA, build_nfa

ANY = frozenset(range(256))


class _Parser:
    def __init__(self, pat: bytes):
        self.p = pat
        self.i = 0

    def peek(self):
        return self.p[self.i] if self.i < len(self.p) else None

    def take(self):
        c = self.p[self.i]
        self.i += 1
        return c

    def parse(self):
        node = self.alt()
        if self.i != len(self.p):
            raise ValueError(f"unexpected {chr(self.p[self.i])!r} at {self.i}")
        return node

    def alt(self):
        parts = [self.concat()]
        while self.peek() == ord("|"):
            self.take()
            parts.append(self.concat())
        return parts[0] if len(parts) == 1 else ("alt", parts)

    def concat(self):
        items = []
        while self.peek() is not None and self.peek() not in (ord("|"), ord(")")):
            items.append(self.repeat())
        return ("cat", items)

    def repeat(self):
        node = self.atom()
        while True:
            c = self.peek()
            if c == ord("*"):
                self.take(); node = ("rep", node, 0, None)
            elif c == ord("+"):
                self.take(); node = ("rep", node, 1, None)
            elif c == ord("?"):
                self.take(); node = ("rep", node, 0, 1)
            elif c == ord("{"):
                self.take()
                j = self.p.index(b"}", self.i)
                body = self.p[self.i:j].decode()
                self.i = j + 1
                if "," in body:
                    lo, hi = body.split(",")
                    node = ("rep", node, int(lo), int(hi) if hi else None)
                else:
                    node = ("rep", node, int(body), int(body))
            else:
                return node

    def atom(self):
        c = self.take()
        if c == ord("("):
            node = self.alt()
            if self.peek() != ord(")"):
                raise ValueError("missing )")
            self.take()
            return node
        if c == ord("["):
            neg = False
            if self.peek() == ord("^"):
                self.take(); neg = True
            members = set()
            first = True
            while first or self.peek() != ord("]"):
                first = False
                a = self.take()
                if a == ord("\\"):
                    a = self.take()
                if self.peek() == ord("-") and self.i + 1 < len(self.p) and self.p[self.i + 1] != ord("]"):
                    self.take()
                    b = self.take()
                    if b == ord("\\"):
                        b = self.take()
                    members.update(range(a, b + 1))
                else:
                    members.add(a)
            self.take()
            return ("set", frozenset(ANY - members if neg else members))
        if c == ord("."):
            return ("set", ANY)
        if c == ord("\\"):
            return ("set", frozenset([self.take()]))
        return ("set", frozenset([c]))


class _Builder:
    def __init__(self):
        self.n = 0
        self.edges: List[Tuple[int, object, int]] = []

    def new(self) -> int:
        self.n += 1
        return self.n - 1

    def frag(self, node) -> Tuple[int, int]:
        kind = node[0]
        if kind == "set":
            s, t = self.new(), self.new()
            self.edges.append((s, node[1], t))
            return s, t
        if kind == "cat":
            s = self.new()
            cur = s
            for item in node[1]:
                a, b = self.frag(item)
                self.edges.append((cur, None, a))
                cur = b
            return s, cur
        if kind == "alt":
            s, t = self.new(), self.new()
            for item in node[1]:
                a, b = self.frag(item)
                self.edges.append((s, None, a))
                self.edges.append((b, None, t))
            return s, t
        if kind == "rep":
            _, sub, lo, hi = node
            s = self.new()
            cur = s
            for _ in range(lo):
                a, b = self.frag(sub)
                self.edges.append((cur, None, a))
                cur = b
            if hi is None:
                a, b = self.frag(sub)
                self.edges.append((cur, None, a))
                self.edges.append((b, None, a))
                t = self.new()
                self.edges.append((cur, None, t))
                self.edges.append((b, None, t))
                return s, t
            t = self.new()
            self.edges.append((cur, None, t))
            for _ in range(hi - lo):
                a, b = self.frag(sub)
                self.edges.append((cur, None, a))
                self.edges.append((b, None, t))
                cur = b
            return s, t
        raise ValueError(kind)


def regex_nfa(patterns: Sequence[Tuple[bytes, int]]) -> NFA:
    """Union of the given (pattern, label) pairs as one epsilon-NFA."""
    b = _Builder()
    q0 = b.new()
    finals = {}
    for pat, label in patterns:
        if isinstance(pat, str):
            pat = pat.encode("latin-1")
        s, t = b.frag(_Parser(pat).parse())
        b.edges.append((q0, None, s))
        finals.setdefault(t, []).append(label)
    class_ids = {}
    classes = []
    src, cls, dst = [], [], []
    for s, k, d in b.edges:
        if k is None:
            c = -1
        else:
            c = class_ids.get(k)
            if c is None:
                c = class_ids[k] = len(classes)
                classes.append(sorted(k))
        src.append(s); cls.append(c); dst.append(d)
    return build_nfa(b.n, q0, src, cls, dst, classes, finals)
