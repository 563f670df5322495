"""CPU checks of the C-ABI library: it loads, exports every symbol include/bae.h declares,
and reports errors loudly (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

import paper_2502_05507_amd as P
from paper_2502_05507_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bae.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bae_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 28
    for n in names:
        assert hasattr(lib, n), n
    # and the binding covers them all
    P.load_library()
    for n in names:
        assert getattr(binding._lib, n).argtypes is not None, n


def test_status_strings_and_table_size():
    lib = P.load_library()
    assert lib.bae_status_string(0) == b"ok"
    assert lib.bae_status_string(-2) == b"invalid geometry"
    assert P.lgf_table_size(0) == 1 and P.lgf_table_size(32) == 33 * 34 * 35 // 6
    assert P.lgf_table_size(-1) == 0


def test_null_arguments_are_rejected():
    lib = P.load_library()
    assert lib.bae_create(None, None, None, None) == -1          # BAE_ERR_ARG
    assert b"null" in lib.bae_last_error()
    assert lib.bae_lgf_table(0.0, -1, None, None) == -1
    assert lib.bae_destroy(None) == 0
