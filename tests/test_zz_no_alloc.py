"""The allocation-free LGF table entry point (bae_lgf_table_noalloc) against the allocating
one (bae_lgf_table) through the C ABI: two calls in a row on the shared static scratch, the
second with a smaller radius, and the radius limit.  Both tables are also held to the
oracle's table (Sec. 2.2), which its own tests pin."""
import numpy as np
import pytest

import paper_2502_05507_amd as P
from oracle import lgf

from gpu_common import device

pytestmark = pytest.mark.gpu


def _tables(s, R):
    import torch
    dev = device()
    E = P.lgf_table_size(R)
    a = torch.full((E,), float("nan"), dtype=torch.float64, device=dev)
    b = torch.full((E,), float("nan"), dtype=torch.float64, device=dev)
    P.lgf_table(s, R, a)
    P.lgf_table_noalloc(s, R, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_table_equals_the_allocating_one():
    # the second call is smaller than the first, the third repeats the second
    results = []
    for s, R in [(0.0488, 96), (0.0, 40), (0.0, 40)]:
        a, b = _tables(s, R)
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b)                       # the same kernels on the same rule
        o = lgf.LGFTable(R, s).values
        assert np.all(np.abs(b - o) <= 1e-13 * np.abs(o) + 1e-17 * o[0])   # the table's own parity bar
        results.append(b)
    assert np.array_equal(results[1], results[2])


def test_noalloc_radius_limit():
    import ctypes
    import torch
    out = torch.empty(8, dtype=torch.float64, device=device())
    lib = P.load_library()
    rc = lib.bae_lgf_table_noalloc(0.0, 2049, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -1 and b"2048" in lib.bae_last_error()
