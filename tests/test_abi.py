"""The C-ABI library loads and exports every entry point include/pfsm.h
declares (no GPU needed: nothing here launches device work)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfsm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pfsm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1110_1716_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1110_1716_amd import build
        build.build()
    return P.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("pfsm_load_dfa", "pfsm_load_nfa", "pfsm_add_pattern", "pfsm_remove_pattern",
              "pfsm_scan", "pfsm_scan_batch"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    import paper_1110_1716_amd as P
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(P.EXPORTS) == set(declared_functions())


def test_strerror_and_argument_errors_without_gpu(lib):
    import paper_1110_1716_amd as P
    assert lib.pfsm_strerror(P.PFSM_EOVERFLOW) == b"more matches than the output capacity"
    # NULL descriptor / NULL handle are rejected on the host, before any HIP call
    assert lib.pfsm_load_dfa(None, None, None) == P.PFSM_EINVAL
    assert lib.pfsm_remove_pattern(None, 0, None) == P.PFSM_EINVAL
    assert lib.pfsm_scan(None, None, 0, None, 0, None, None) == P.PFSM_EINVAL
    assert b"NULL" in lib.pfsm_last_error()
