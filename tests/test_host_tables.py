"""Host logic of pattern edits, on the CPU: the library's NFA table builder
(csrc/nfa_host.cpp), compiled with g++ against a stand-in HIP runtime
(tests/hostsim), loads an NFA and applies adds, removes and pair-cache
switches.  After every step a plain simulation that follows only the packed
tables, the way the scan kernel reads them, must report exactly the oracle's
matches of the edited union (Section III.A: the union's matches are those of
its parts; a removed label is no longer reported; a removed added pattern is
cut off entirely), and must never index outside an array."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from workloads.regex import regex_nfa

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("hostsim") / "nfa_tables_sim")
    cmd = [gxx, "-std=c++17", "-O2", "-w", "-I", os.path.join(HERE, "hostsim"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1110_1716_amd", "csrc"), os.path.join(HERE, "hostsim", "nfa_tables_sim.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def write_desc(f, a):
    f.write(f"{a.n_states} {a.q0} {a.n_classes}\n")
    for arr in (a.row_ptr, a.edge_class, a.edge_dst, a.class_bits, a.final_off, a.final_labels):
        f.write(" ".join(str(int(v)) for v in np.asarray(arr).ravel()) + "\n")


def relabel(a, base):
    return W.NFA(a.n_states, a.q0, a.n_classes, a.row_ptr, a.edge_class, a.edge_dst, a.class_bits, a.final_off,
                 np.asarray(a.final_labels) + base)


def labels_of(a):
    return sorted(set(int(v) for v in np.asarray(a.final_labels)))


def expected(base, disabled, added, x):
    """Oracle matches of the union: the loaded NFA without its disabled
    labels, plus every added pattern still present."""
    ref, _ = oracle.scan(base, x)
    ref = np.asarray(ref).reshape(-1, 3)
    parts = [ref[~np.isin(ref[:, 2], list(disabled))]] if len(ref) else [ref]
    for p in added:
        r, _ = oracle.scan(p, x)
        parts.append(np.asarray(r).reshape(-1, 3))
    allm = np.concatenate(parts) if parts else np.zeros((0, 3), np.int32)
    return sorted(set(map(tuple, allm.tolist())))


def run_case(sim, tmp_path, base, ops_gen, x, rng, min_gap_chains=0):
    """ops_gen yields ('a', nfa) / ('r', label) / ('k', 0|1); returns the
    number of steps checked.  The simulator also checks, after every step,
    that each gap the scan finishes in one pass heads a simple chain; at
    least min_gap_chains of them must have been seen at some step."""
    path, out = tmp_path / "case.txt", tmp_path / "out.txt"
    ops = list(ops_gen)
    with open(path, "w") as f:
        write_desc(f, base)
        f.write(f"{len(x)}\n" + " ".join(str(int(v)) for v in x) + "\n")
        for op in ops:
            if op[0] == "a":
                f.write("a\n")
                write_desc(f, op[1])
            else:
                f.write(f"{op[0]} {op[1]}\n")
    r = subprocess.run([sim, str(path), str(out)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    seen = [int(l.split()[-1]) for l in r.stderr.splitlines() if l.startswith("gap chains")]
    assert max(seen, default=0) >= min_gap_chains, seen
    blocks = open(out).read().split("== ")[1:]
    assert len(blocks) == len(ops) + 1
    # replay the edits on the reference side
    disabled, added, cut = set(), [], set()
    base_labels = set(labels_of(base))
    for step, blk in enumerate(blocks):
        lines = blk.strip().split("\n")
        rc = int(lines[0])
        if step > 0:
            op = ops[step - 1]
            if op[0] == "a":
                present = (base_labels - disabled) | {l for i, p in enumerate(added) if i not in cut
                                                      for l in labels_of(p)}
                want = -6 if set(labels_of(op[1])) & present else 0
                assert rc == want, (step, op[0], rc)
                if rc == 0:
                    added.append(op[1])
            elif op[0] == "r":
                lab = op[1]
                hit = False
                if lab in base_labels and lab not in disabled:
                    disabled.add(lab)
                    hit = True
                for i, p in enumerate(added):
                    if i not in cut and lab in labels_of(p):
                        cut.add(i)
                        hit = True
                assert rc == (0 if hit else -5), (step, lab, rc)
            else:
                assert rc == 0
        else:
            assert rc == 0
        got = [tuple(int(v) for v in ln.split()) for ln in lines[1:] if ln]
        want = expected(base, disabled, [p for i, p in enumerate(added) if i not in cut], x)
        assert got == want, (step, ops[step - 1][0] if step else "load", len(got), len(want))
    return len(blocks)


def random_ops(rng, base, n_ops):
    present = labels_of(base)
    nxt = 1000
    for _ in range(n_ops):
        r = rng.random()
        if r < 0.45:
            if rng.random() < 0.5:
                sig = W.signature_union(rng, 1, len_lo=3, len_hi=6, frac_gap=0.3, gap_max=4, label_base=nxt)
                pat = W.union_nfa(sig, gap_max=4)
                pat = W.NFA(pat.n_states, pat.q0, pat.n_classes, pat.row_ptr, pat.edge_class, pat.edge_dst,
                            _fold_to(pat.class_bits, b"abcde"), pat.final_off, pat.final_labels)
            else:
                pat = relabel(W.random_nfa(rng, int(rng.integers(2, 9)), list(b"abcde"), int(rng.integers(2, 16)),
                                           n_labels=3), nxt)
            if not labels_of(pat):
                continue
            if present and rng.random() < 0.1:  # a label already present: refused
                pat = relabel(pat, present[0] - int(np.asarray(pat.final_labels).min()))
            else:
                present += labels_of(pat)
                nxt += 10
            yield ("a", pat)
        elif r < 0.85:
            if present and rng.random() < 0.9:
                yield ("r", present.pop(int(rng.integers(0, len(present)))))
            else:
                yield ("r", 987654)  # never present
        else:
            yield ("k", int(rng.integers(0, 2)))


def _fold_to(class_bits, alphabet):
    """Restrict byte classes to the input alphabet, keeping each class
    non-empty (single bytes map onto the alphabet), so that random
    signatures can match the random inputs."""
    bits = np.asarray(class_bits, dtype=np.uint32).reshape(-1, 8).copy()
    al = np.frombuffer(alphabet, np.uint8)
    out = np.zeros_like(bits)
    for k in range(bits.shape[0]):
        members = [b for b in range(256) if (bits[k, b >> 5] >> (b & 31)) & 1]
        if len(members) == 256:
            out[k] = bits[k]
            continue
        for b in members:
            a = int(al[b % len(al)])
            out[k, a >> 5] |= np.uint32(1 << (a & 31))
    return out.ravel()


@pytest.mark.parametrize("seed", range(24))
def test_random_unions_and_edits(sim, tmp_path, seed):
    rng = np.random.default_rng(700 + seed)
    kind = seed % 4
    if kind == 0:  # a union of signature chains under an ancillary initial state
        sigs = W.signature_union(rng, int(rng.integers(3, 25)), len_lo=3, len_hi=7, frac_gap=0.2, gap_max=4)
        base = W.union_nfa(sigs, gap_max=4)
        base = W.NFA(base.n_states, base.q0, base.n_classes, base.row_ptr, base.edge_class, base.edge_dst,
                     _fold_to(base.class_bits, b"abcde"), base.final_off, base.final_labels)
    elif kind == 1:  # one connected random NFA (no ancillary state)
        base = W.random_nfa(rng, int(rng.integers(3, 20)), list(b"abcde"), int(rng.integers(3, 40)))
    elif kind == 2:
        pats = [(b"[a-d]*e", 0), (b"ab(c|d)+", 1), (b"a.{0,3}b", 2), (b"(ab|cd)*e", 3), (b"d[ab]c", 4)]
        base = regex_nfa(pats[:int(rng.integers(1, len(pats) + 1))])
    else:
        base = W.dfa_as_nfa(W.random_dfa(rng, int(rng.integers(2, 10)), 5, p_dead=0.3, n_finals=3))
        if base.n_classes:  # its classes are symbols 0-4: map them to a-e
            base = W.NFA(base.n_states, base.q0, base.n_classes, base.row_ptr, base.edge_class, base.edge_dst,
                         _fold_to(base.class_bits, b"abcde"), base.final_off, base.final_labels)
    x = rng.choice(np.frombuffer(b"abcde", np.uint8), int(rng.integers(50, 260)))
    steps = run_case(sim, tmp_path, base, random_ops(rng, base, int(rng.integers(2, 10))), x, rng)
    assert steps >= 1


def test_signature_union_many_edits(sim, tmp_path):
    """A 300-signature union (cfg4's recipe) over a 4-letter input with 40
    alternating adds and removes; one add is large enough to move the
    tables to new buffers."""
    rng = np.random.default_rng(77)
    sigs = W.signature_union(rng, 300, len_lo=3, len_hi=6, frac_gap=0.05, gap_max=8)
    base = W.union_nfa(sigs, gap_max=8)
    base = W.NFA(base.n_states, base.q0, base.n_classes, base.row_ptr, base.edge_class, base.edge_dst,
                 _fold_to(base.class_bits, b"abcd"), base.final_off, base.final_labels)
    ops, present, nxt = [], [s.label for s in sigs], 5000
    for i in range(40):
        if i % 2 == 0:
            n = 200 if i == 20 else 1
            sig = W.signature_union(rng, n, len_lo=3, len_hi=6, frac_gap=0.1, gap_max=8, label_base=nxt)
            pat = W.union_nfa(sig, gap_max=8)
            pat = W.NFA(pat.n_states, pat.q0, pat.n_classes, pat.row_ptr, pat.edge_class, pat.edge_dst,
                        _fold_to(pat.class_bits, b"abcd"), pat.final_off, pat.final_labels)
            ops.append(("a", pat))
            present += labels_of(pat)
            nxt += n
        else:
            ops.append(("r", present.pop(int(rng.integers(0, len(present))))))
    x = rng.choice(np.frombuffer(b"abcd", np.uint8), 400)
    assert run_case(sim, tmp_path, base, iter(ops), x, rng, min_gap_chains=1) == 41
