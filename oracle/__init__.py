"""CPU oracle for the all-matches PFSM scan.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the GPU library
and its binding) never does, and the two share no code.

Contents:

* ``scan``      -- the plain definition of the match set, in C
                   (``pfsm_oracle.c``), per start position, multi-threaded.
* ``brute``     -- the same definition evaluated substring by substring in
                   pure Python (tiny inputs only).
* ``tagset``    -- the paper's own algorithm (Section III.B: tagged
                   reinitialisation and the four steps per symbol), pure
                   Python, with its online reporting order (Fig. 2).
* ``subset``    -- subset construction of an NFA into a DFA whose final
                   states carry label sets (Section II), for the invariant
                   "NFA and its DFA report the same matches".
* ``compose``   -- the union through an ancillary initial state
                   (Section III.A) and label removal, on descriptors.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

from . import brute, compose, subset, tagset  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pfsm_oracle.c")
_LIB = os.path.join(_HERE, "libpfsm_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle in place with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.pfsm_oracle_dfa.restype = i64
        lib.pfsm_oracle_dfa.argtypes = [i32, i32, i32, p, p, p, p, p, i64, i64, i64, i32, i32,
                                        ctypes.POINTER(ctypes.c_void_p), p]
        lib.pfsm_oracle_nfa.restype = i64
        lib.pfsm_oracle_nfa.argtypes = [i32, i32, i32, p, p, p, p, p, p, p, i64, i64, i64, i32,
                                        i32, i32, ctypes.POINTER(ctypes.c_void_p), p]
        lib.pfsm_oracle_free.restype = None
        lib.pfsm_oracle_free.argtypes = [p]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def scan(fsm, x, s_lo: int = 0, s_hi: Optional[int] = None, prune: bool = True,
         memo: bool = True, threads: Optional[int] = None) -> Tuple[np.ndarray, Dict[str, int]]:
    """All matches of ``fsm`` (a workloads DFA or NFA) in ``x``.

    Returns (int32 array [m, 3] of (start, end, label) sorted by (start, end,
    label), {"T": instance-steps, "X": state activations}).  Only starts in
    [s_lo, s_hi) are reported; their walks read the whole remaining input.
    """
    lib = _load()
    x = np.ascontiguousarray(np.frombuffer(bytes(x), np.uint8) if isinstance(x, (bytes, bytearray))
                             else x, dtype=np.uint8)
    n = x.size
    if s_hi is None:
        s_hi = n
    if threads is None:
        threads = default_threads()
    out = ctypes.c_void_p()
    work = np.zeros(2, np.int64)
    keep = []

    def c(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    if fsm.kind == "dfa":
        b2s = None if fsm.byte_to_symbol is None else c(fsm.byte_to_symbol, np.int16)
        cnt = lib.pfsm_oracle_dfa(fsm.n_states, fsm.n_symbols, fsm.q0, _ptr(b2s),
                                  _ptr(c(fsm.delta, np.int32)), _ptr(c(fsm.final_off, np.int32)),
                                  _ptr(c(fsm.final_labels, np.int32)), _ptr(x), n, s_lo, s_hi,
                                  int(prune), threads, ctypes.byref(out), _ptr(work))
    else:
        cnt = lib.pfsm_oracle_nfa(fsm.n_states, fsm.q0, fsm.n_classes,
                                  _ptr(c(fsm.row_ptr, np.int32)), _ptr(c(fsm.edge_class, np.int32)),
                                  _ptr(c(fsm.edge_dst, np.int32)), _ptr(c(fsm.class_bits, np.uint32)),
                                  _ptr(c(fsm.final_off, np.int32)), _ptr(c(fsm.final_labels, np.int32)),
                                  _ptr(x), n, s_lo, s_hi, int(prune), int(memo), threads,
                                  ctypes.byref(out), _ptr(work))
    if cnt == -1:
        raise ValueError("oracle: invalid automaton descriptor")
    if cnt < 0:
        raise MemoryError("oracle: out of memory")
    try:
        if cnt:
            buf = (ctypes.c_int32 * (3 * cnt)).from_address(out.value)
            res = np.frombuffer(buf, dtype=np.int32).reshape(cnt, 3).copy()
        else:
            res = np.zeros((0, 3), np.int32)
    finally:
        if out.value:
            lib.pfsm_oracle_free(out)
    return res, {"T": int(work[0]), "X": int(work[1])}
