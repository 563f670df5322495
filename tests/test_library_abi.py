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
    assert lib.bae_lgf_table_noalloc(0.0, 8, None, None) == -1
    assert lib.bae_lgf_sum_repeat(None, None, 1, 1, 1, None) == -1
    assert lib.bae_destroy(None) == 0


@pytest.mark.parametrize("n,h,sigma,what", [((2050, 5, 5), 1 / 16, 0.0, "2049"), ((5, 4, 5), 1 / 16, 0.0, "2049"),
                                            ((17, 17, 17), 0.0, 0.0, "h"), ((17, 17, 17), 1 / 16, -1.0, "sigma")])
def test_grid_is_validated_before_any_device_work(n, h, sigma, what):
    # n in [5, 2049]: lattice coordinates up to 2048 are exact in binary16, which the FP32
    # far field's packed differences rely on
    with pytest.raises(P.BaeError) as e:
        P.Context(n, h, (0, 0, 0), sigma, "sphere", (0.5, 0.5, 0.5), (0.4,))
    assert e.value.status == -1
    assert what in str(e.value)
