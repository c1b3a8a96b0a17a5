"""Python binding of libpfsm (include/pfsm.h): an all-matches Parallel Finite
State Machine scanner for MI355X (gfx950).

The binding only marshals arguments: descriptors are passed as numpy arrays
(any object with the descriptor's attribute names works, e.g. the ``DFA`` and
``NFA`` dataclasses of the ``workloads`` package), device buffers as torch
tensors, streams as ``torch.cuda.Stream`` (default: the current stream).
Every step of a scan runs in the library's HIP kernels; when libpfsm.so is
missing, loading fails loudly -- there is no fallback.

Names follow the C ABI: ``pfsm_load_dfa``, ``pfsm_load_nfa``,
``pfsm_add_pattern``, ``pfsm_remove_pattern``, ``pfsm_scan``,
``pfsm_scan_async``, ``pfsm_scan_noalloc``, ``pfsm_scan_batch``, ``pfsm_scan_batch_async``, ``pfsm_last_stats``,
``pfsm_free``; ``Stream`` wraps ``pfsm_stream_*`` and ``Server`` ``pfsm_server_*``.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfsm.so")

PFSM_OK = 0
PFSM_EINVAL = -1
PFSM_ENOMEM = -2
PFSM_EOVERFLOW = -3
PFSM_EHIP = -4
PFSM_ENOENT = -5
PFSM_EEXIST = -6
PFSM_ENOSYS = -7

PFSM_OPT_SEGMENT = 1
PFSM_OPT_WORKGROUPS_PER_CU = 2
PFSM_OPT_TABLE_BUDGET = 3
PFSM_OPT_PAIR_CACHE = 4
PFSM_OPT_MAX_WORKGROUPS_PER_CU = 5
PFSM_OPT_RESIDENT_TABLE = 6
PFSM_OPT_MERGED_WALKS = 7
PFSM_OPT_MERGED_COUNT_LIMIT = 8
PFSM_OPT_LAYOUT_EPOCH = 9

# Exported symbols of libpfsm.so, as declared in include/pfsm.h.
EXPORTS = ("pfsm_load_dfa", "pfsm_load_nfa", "pfsm_add_pattern", "pfsm_remove_pattern", "pfsm_scan",
           "pfsm_scan_async", "pfsm_scan_batch", "pfsm_scan_batch_async", "pfsm_last_stats", "pfsm_free",
           "pfsm_strerror", "pfsm_last_error", "pfsm_server_create", "pfsm_server_submit", "pfsm_server_submit_borrowed",
           "pfsm_server_wait",
           "pfsm_server_times", "pfsm_server_release", "pfsm_server_stats_get", "pfsm_server_destroy",
           "pfsm_stream_open", "pfsm_stream_feed", "pfsm_stream_info", "pfsm_stream_close",
           "pfsm_set_option", "pfsm_get_option", "pfsm_tune", "pfsm_release_cached", "pfsm_scan_noalloc")


class PfsmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class _DfaDesc(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("n_symbols", ctypes.c_int32), ("q0", ctypes.c_int32),
                ("byte_to_symbol", ctypes.c_void_p), ("delta", ctypes.c_void_p),
                ("final_off", ctypes.c_void_p), ("final_labels", ctypes.c_void_p)]


class _NfaDesc(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("q0", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("edge_class", ctypes.c_void_p),
                ("edge_dst", ctypes.c_void_p), ("class_bits", ctypes.c_void_p),
                ("final_off", ctypes.c_void_p), ("final_labels", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("transitions", ctypes.c_int64), ("activations", ctypes.c_int64),
                ("matches", ctypes.c_int64), ("long_walks", ctypes.c_int64)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("segment", ctypes.c_int64), ("workgroups_per_cu", ctypes.c_int64),
                ("table_budget", ctypes.c_int64), ("pair_cache", ctypes.c_int64),
                ("ms_before", ctypes.c_double), ("ms_after", ctypes.c_double),
                ("configs", ctypes.c_int32), ("pad", ctypes.c_int32), ("matches", ctypes.c_int64),
                ("merged_walks", ctypes.c_int64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("reruns", ctypes.c_int64), ("requests", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("matches", ctypes.c_int64), ("peak_inflight", ctypes.c_int64),
                ("pack_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64), ("deliver_ns", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpfsm.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpfsm.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "pfsm_load_dfa": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(_DfaDesc), vp]),
        "pfsm_load_nfa": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(_NfaDesc), vp]),
        "pfsm_add_pattern": (ctypes.c_int, [vp, ctypes.POINTER(_NfaDesc), vp]),
        "pfsm_remove_pattern": (ctypes.c_int, [vp, i32, vp]),
        "pfsm_scan": (ctypes.c_int, [vp, vp, i64, vp, i64, ctypes.POINTER(i64), vp]),
        "pfsm_scan_async": (ctypes.c_int, [vp, vp, i64, vp, i64, vp, vp]),
        "pfsm_scan_noalloc": (ctypes.c_int, [vp, vp, i64, vp, i64, vp, vp]),
        "pfsm_scan_batch": (ctypes.c_int, [vp, i32, vp, vp, vp, i32, vp, i64, vp,
                                           ctypes.POINTER(i64), vp]),
        "pfsm_scan_batch_async": (ctypes.c_int, [vp, i32, vp, vp, vp, i32, vp, i64, vp, vp]),
        "pfsm_last_stats": (ctypes.c_int, [vp, ctypes.POINTER(_Stats), vp]),
        "pfsm_free": (None, [vp]),
        "pfsm_release_cached": (None, []),
        "pfsm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "pfsm_server_create": (ctypes.c_int, [ctypes.POINTER(vp), vp, i32, i64, i32]),
        "pfsm_server_submit": (ctypes.c_int, [vp, i32, vp, i64, ctypes.POINTER(i64)]),
        "pfsm_server_submit_borrowed": (ctypes.c_int, [vp, i32, vp, i64, ctypes.POINTER(i64)]),
        "pfsm_server_wait": (ctypes.c_int, [vp, i64, ctypes.POINTER(vp), ctypes.POINTER(i64)]),
        "pfsm_server_times": (ctypes.c_int, [vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "pfsm_server_release": (ctypes.c_int, [vp, i64]),
        "pfsm_server_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(_ServerStats)]),
        "pfsm_server_destroy": (None, [vp]),
        "pfsm_last_error": (ctypes.c_char_p, []),
        "pfsm_stream_open": (ctypes.c_int, [ctypes.POINTER(vp), vp]),
        "pfsm_stream_feed": (ctypes.c_int, [vp, vp, i64, vp, i64, ctypes.POINTER(i64), vp]),
        "pfsm_stream_info": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp]),
        "pfsm_stream_close": (None, [vp]),
        "pfsm_set_option": (ctypes.c_int, [vp, i32, i64, vp]),
        "pfsm_get_option": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64)]),
        "pfsm_tune": (ctypes.c_int, [vp, vp, i64, i32, ctypes.POINTER(_TuneReport), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    atexit.register(_release_at_exit)
    return lib


# Objects still open when the interpreter exits are released by an atexit
# hook, in dependency order (servers, then streams, then handles, then the
# library's cached batch buffers), while the HIP runtime is still up: never
# from finalizers that run in no set order during shutdown.
_live_servers: "weakref.WeakSet" = weakref.WeakSet()
_live_streams: "weakref.WeakSet" = weakref.WeakSet()
_live_handles: "weakref.WeakSet" = weakref.WeakSet()


def _release_at_exit():
    for group in (_live_servers, _live_streams, _live_handles):
        for obj in list(group):
            try:
                obj.close() if hasattr(obj, "close") else obj.free()
            except Exception:
                pass
    if _lib is not None:
        _lib.pfsm_release_cached()


def _check(rc: int):
    if rc != PFSM_OK:
        lib = load_library()
        raise PfsmError(rc, lib.pfsm_last_error().decode() or lib.pfsm_strerror(rc).decode())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _arr(a, dt, keep):
    a = np.ascontiguousarray(a, dtype=dt)
    keep.append(a)
    return a.ctypes.data


def _dfa_desc(d, keep) -> _DfaDesc:
    b2s = None if d.byte_to_symbol is None else _arr(d.byte_to_symbol, np.int16, keep)
    return _DfaDesc(int(d.n_states), int(d.n_symbols), int(d.q0), b2s, _arr(d.delta, np.int32, keep),
                    _arr(d.final_off, np.int32, keep), _arr(d.final_labels, np.int32, keep))


def _nfa_desc(a, keep) -> _NfaDesc:
    return _NfaDesc(int(a.n_states), int(a.q0), int(a.n_classes), _arr(a.row_ptr, np.int32, keep),
                    _arr(a.edge_class, np.int32, keep), _arr(a.edge_dst, np.int32, keep),
                    _arr(a.class_bits, np.uint32, keep), _arr(a.final_off, np.int32, keep),
                    _arr(a.final_labels, np.int32, keep))


class Pfsm:
    """A loaded automaton (owns the C handle)."""

    def __init__(self, ptr: int, kind: str):
        self._ptr = ptr
        self.kind = kind
        _live_handles.add(self)

    @property
    def ptr(self) -> int:
        if not self._ptr:
            raise PfsmError(PFSM_EINVAL, "handle already freed")
        return self._ptr

    def free(self):
        if self._ptr:
            load_library().pfsm_free(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pfsm_load_dfa(dfa, stream=None) -> Pfsm:
    lib = load_library()
    keep = []
    desc = _dfa_desc(dfa, keep)
    h = ctypes.c_void_p()
    _check(lib.pfsm_load_dfa(ctypes.byref(h), ctypes.byref(desc), _stream_ptr(stream)))
    return Pfsm(h.value, "dfa")


def pfsm_load_nfa(nfa, stream=None) -> Pfsm:
    lib = load_library()
    keep = []
    desc = _nfa_desc(nfa, keep)
    h = ctypes.c_void_p()
    _check(lib.pfsm_load_nfa(ctypes.byref(h), ctypes.byref(desc), _stream_ptr(stream)))
    return Pfsm(h.value, "nfa")


def pfsm_load(automaton, stream=None) -> Pfsm:
    return (pfsm_load_dfa if automaton.kind == "dfa" else pfsm_load_nfa)(automaton, stream)


def pfsm_add_pattern(h: Pfsm, pattern, stream=None) -> None:
    keep = []
    desc = _nfa_desc(pattern, keep)
    _check(load_library().pfsm_add_pattern(h.ptr, ctypes.byref(desc), _stream_ptr(stream)))


def pfsm_remove_pattern(h: Pfsm, label: int, stream=None) -> None:
    _check(load_library().pfsm_remove_pattern(h.ptr, int(label), _stream_ptr(stream)))


def _check_input(x):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.uint8 and x.dim() == 1):
        raise PfsmError(PFSM_EINVAL, "input must be a 1-D uint8 CUDA tensor")
    if not x.is_contiguous():
        raise PfsmError(PFSM_EINVAL, "input must be contiguous")


def _check_out(out):
    import torch
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.int32
            and out.dim() == 2 and out.shape[1] == 3 and out.is_contiguous()):
        raise PfsmError(PFSM_EINVAL, "out must be a contiguous [cap, 3] int32 CUDA tensor")


def pfsm_scan(h: Pfsm, x, out=None, stream=None, cap: Optional[int] = None) -> Tuple[int, "torch.Tensor"]:
    """Scan device bytes ``x``; returns (n_matches, out[:n_matches]).

    With ``out=None`` an output of ``cap`` rows (default: n/16 + 1024) is
    allocated and grown once when the scan reports overflow.  With a given
    ``out`` too small for the result, PfsmError(PFSM_EOVERFLOW) is raised.
    """
    import torch
    _check_input(x)
    lib = load_library()
    st = _stream_ptr(stream)
    auto = out is None
    if auto:
        cap = cap if cap is not None else x.numel() // 16 + 1024
        out = torch.empty((cap, 3), dtype=torch.int32, device=x.device)
    _check_out(out)
    n = ctypes.c_int64()
    rc = lib.pfsm_scan(h.ptr, x.data_ptr(), x.numel(), out.data_ptr(), out.shape[0], ctypes.byref(n), st)
    if rc == PFSM_EOVERFLOW and auto:
        out = torch.empty((n.value, 3), dtype=torch.int32, device=x.device)
        rc = lib.pfsm_scan(h.ptr, x.data_ptr(), x.numel(), out.data_ptr(), out.shape[0], ctypes.byref(n), st)
    _check(rc)
    return n.value, out[:n.value]


def pfsm_scan_async(h: Pfsm, x, out, d_n_matches, stream=None) -> None:
    """Enqueue a scan; the total goes to the int64 CUDA tensor ``d_n_matches``."""
    import torch
    _check_input(x)
    _check_out(out)
    if not (isinstance(d_n_matches, torch.Tensor) and d_n_matches.is_cuda and d_n_matches.dtype == torch.int64):
        raise PfsmError(PFSM_EINVAL, "d_n_matches must be an int64 CUDA tensor")
    _check(load_library().pfsm_scan_async(h.ptr, x.data_ptr(), x.numel(), out.data_ptr(), out.shape[0],
                                          d_n_matches.data_ptr(), _stream_ptr(stream)))


def pfsm_scan_noalloc(h: Pfsm, x, out, d_n_matches, stream=None) -> None:
    """pfsm_scan_async through the entry point that allocates nothing (DFA handles)."""
    import torch
    _check_input(x)
    _check_out(out)
    if not (isinstance(d_n_matches, torch.Tensor) and d_n_matches.is_cuda and d_n_matches.dtype == torch.int64):
        raise PfsmError(PFSM_EINVAL, "d_n_matches must be an int64 CUDA tensor")
    _check(load_library().pfsm_scan_noalloc(h.ptr, x.data_ptr(), x.numel(), out.data_ptr(), out.shape[0],
                                            d_n_matches.data_ptr(), _stream_ptr(stream)))


def pfsm_scan_batch(handles, data, stream_off, stream_automaton, out=None, match_off=None, stream=None,
                    cap: Optional[int] = None):
    """Scan many streams, each against one of ``handles``, in one call.

    ``data``: 1-D uint8 CUDA tensor holding every stream; ``stream_off``:
    int64 CUDA tensor [n_streams + 1] of byte offsets into it;
    ``stream_automaton``: int32 CUDA tensor [n_streams] of indices into
    ``handles``.  Returns (n_matches, out[:n_matches], match_off): matches
    grouped by stream in stream order, positions relative to each stream's
    first byte, group g at out[match_off[g]:match_off[g + 1]].  With
    ``out=None`` an output of ``cap`` rows is allocated and grown once on
    overflow.
    """
    import torch
    _check_input(data)
    n_streams = stream_automaton.numel()
    for t, dt, name in ((stream_off, torch.int64, "stream_off"), (stream_automaton, torch.int32, "stream_automaton")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.dim() == 1 and t.is_contiguous()):
            raise PfsmError(PFSM_EINVAL, f"{name} must be a contiguous 1-D {dt} CUDA tensor")
    if stream_off.numel() != n_streams + 1:
        raise PfsmError(PFSM_EINVAL, "stream_off must have n_streams + 1 entries")
    lib = load_library()
    st = _stream_ptr(stream)
    if match_off is None:
        match_off = torch.empty(n_streams + 1, dtype=torch.int64, device=data.device)
    auto = out is None
    if auto:
        cap = cap if cap is not None else data.numel() // 16 + 1024
        out = torch.empty((cap, 3), dtype=torch.int32, device=data.device)
    _check_out(out)
    arr = (ctypes.c_void_p * len(handles))(*[h.ptr for h in handles])
    n = ctypes.c_int64()

    def call(o):
        return lib.pfsm_scan_batch(arr, len(handles), data.data_ptr(), stream_off.data_ptr(),
                                   stream_automaton.data_ptr(), n_streams, o.data_ptr(), o.shape[0],
                                   match_off.data_ptr(), ctypes.byref(n), st)

    rc = call(out)
    if rc == PFSM_EOVERFLOW and auto:
        out = torch.empty((n.value, 3), dtype=torch.int32, device=data.device)
        rc = call(out)
    _check(rc)
    return n.value, out[:n.value], match_off


def pfsm_scan_batch_async(handles, data, stream_off, stream_automaton, out, match_off, stream=None) -> None:
    """Enqueue a batch with no host round trip (capturable in a HIP graph);
    the total is match_off[n_streams].  Buffers must have been sized by a
    pfsm_scan_batch call of the same or larger size on the same stream.
    A captured graph sees later pattern edits of its handles while their
    PFSM_OPT_LAYOUT_EPOCH option is unchanged; after it changes, the graph
    still replays safely but scans the automaton of before the change:
    run pfsm_scan_batch once and capture again."""
    _check_input(data)
    _check_out(out)
    arr = (ctypes.c_void_p * len(handles))(*[h.ptr for h in handles])
    _check(load_library().pfsm_scan_batch_async(arr, len(handles), data.data_ptr(), stream_off.data_ptr(),
                                                stream_automaton.data_ptr(), stream_automaton.numel(),
                                                out.data_ptr(), out.shape[0], match_off.data_ptr(),
                                                _stream_ptr(stream)))


def pfsm_last_stats(h: Pfsm, stream=None) -> dict:
    s = _Stats()
    _check(load_library().pfsm_last_stats(h.ptr, ctypes.byref(s), _stream_ptr(stream)))
    return {"transitions": s.transitions, "activations": s.activations, "matches": s.matches,
            "long_walks": s.long_walks}


def pfsm_free(h: Pfsm) -> None:
    h.free()


def pfsm_set_option(h: Pfsm, option: int, value: int, stream=None) -> None:
    _check(load_library().pfsm_set_option(h.ptr, int(option), int(value), _stream_ptr(stream)))


def pfsm_get_option(h: Pfsm, option: int) -> int:
    v = ctypes.c_int64()
    _check(load_library().pfsm_get_option(h.ptr, int(option), ctypes.byref(v)))
    return v.value


def pfsm_tune(h: Pfsm, sample, reps: int = 10, stream=None) -> dict:
    """Autotune h's launch settings on device bytes ``sample``; returns the
    report (settings kept, ms per scan before and after, settings timed)."""
    _check_input(sample)
    r = _TuneReport()
    _check(load_library().pfsm_tune(h.ptr, sample.data_ptr(), sample.numel(), int(reps), ctypes.byref(r),
                                    _stream_ptr(stream)))
    return {f: getattr(r, f) for f, _ in _TuneReport._fields_ if f != "pad"}


class Stream:
    """A byte stream scanned piece by piece (include/pfsm.h, pfsm_stream_*):
    the matches reported by all feeds together are those of one pfsm_scan of
    the concatenated pieces; each feed reports the matches ending inside its
    piece, positions counted from the stream's first byte."""

    def __init__(self, h: Pfsm):
        p = ctypes.c_void_p()
        _check(load_library().pfsm_stream_open(ctypes.byref(p), h.ptr))
        self._h = h
        self._ptr = p.value
        _live_streams.add(self)

    def feed(self, x, out=None, stream=None, cap: Optional[int] = None) -> Tuple[int, "torch.Tensor"]:
        """Feed device bytes ``x``; returns (n_matches, out[:n_matches]).
        Output handling as in pfsm_scan (an automatic buffer is grown once)."""
        import torch
        _check_input(x)
        lib = load_library()
        st = _stream_ptr(stream)
        auto = out is None
        if auto:
            cap = cap if cap is not None else x.numel() // 16 + 1024
            out = torch.empty((cap, 3), dtype=torch.int32, device=x.device)
        _check_out(out)
        n = ctypes.c_int64()
        rc = lib.pfsm_stream_feed(self._ptr, x.data_ptr(), x.numel(), out.data_ptr(), out.shape[0],
                                  ctypes.byref(n), st)
        if rc == PFSM_EOVERFLOW and auto:
            out = torch.empty((n.value, 3), dtype=torch.int32, device=x.device)
            rc = lib.pfsm_stream_feed(self._ptr, x.data_ptr(), x.numel(), out.data_ptr(), out.shape[0],
                                      ctypes.byref(n), st)
        _check(rc)
        return n.value, out[:n.value]

    def info(self, stream=None) -> Tuple[int, int]:
        """(bytes fed so far, live instances carried into the next piece)."""
        pos, car = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().pfsm_stream_info(self._ptr, ctypes.byref(pos), ctypes.byref(car), _stream_ptr(stream)))
        return pos.value, car.value

    def close(self):
        if getattr(self, "_ptr", None):
            load_library().pfsm_stream_close(self._ptr)
            self._ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching scan server over resident handles (include/pfsm.h,
    pfsm_server_*).  Requests are host byte strings; results are
    int32 [k, 3] arrays of (start, end, label), ascending."""

    def __init__(self, handles, mem_budget: int = 1 << 30, max_batch: int = 4096):
        lib = load_library()
        self._handles = list(handles)
        arr = (ctypes.c_void_p * len(self._handles))(*[h.ptr for h in self._handles])
        p = ctypes.c_void_p()
        _check(lib.pfsm_server_create(ctypes.byref(p), arr, len(self._handles), int(mem_budget), int(max_batch)))
        self._ptr = p.value
        _live_servers.add(self)

    def submit(self, automaton: int, data, borrow: bool = False) -> int:
        """Queue a request.  With borrow=True the server reads ``data`` (a
        contiguous uint8 array) in place: keep it unchanged until wait()."""
        a = np.ascontiguousarray(np.frombuffer(data, np.uint8) if isinstance(data, (bytes, bytearray))
                                 else np.asarray(data, np.uint8))
        rid = ctypes.c_int64()
        fn = load_library().pfsm_server_submit_borrowed if borrow else load_library().pfsm_server_submit
        _check(fn(self._ptr, int(automaton), a.ctypes.data if a.size else None, a.size, ctypes.byref(rid)))
        return rid.value

    def times(self, rid: int) -> Tuple[int, int]:
        """(submitted, finished) in CLOCK_MONOTONIC ns (time.monotonic_ns)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().pfsm_server_times(self._ptr, int(rid), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def wait(self, rid: int, release: bool = True) -> np.ndarray:
        lib = load_library()
        ptr, n = ctypes.c_void_p(), ctypes.c_int64()
        _check(lib.pfsm_server_wait(self._ptr, int(rid), ctypes.byref(ptr), ctypes.byref(n)))
        k = n.value
        out = (np.frombuffer((ctypes.c_int32 * (3 * k)).from_address(ptr.value), np.int32).reshape(k, 3).copy()
               if k else np.zeros((0, 3), np.int32))
        if release:
            _check(lib.pfsm_server_release(self._ptr, int(rid)))
        return out

    def release(self, rid: int) -> None:
        """Drop a finished request (after wait(rid, release=False))."""
        _check(load_library().pfsm_server_release(self._ptr, int(rid)))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(load_library().pfsm_server_stats_get(self._ptr, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_ptr", None):
            load_library().pfsm_server_destroy(self._ptr)
            self._ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
