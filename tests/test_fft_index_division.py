"""The index division of the LDS FFT kernels, checked exhaustively on the CPU.

The FFT stages and the line kernels split a flat element index e into (line, position) by
truncating e * r, where r is the hardware float reciprocal of d (accurate to one ulp) scaled by
1 + 2^-16, with no correction step.  The kernels rely on this being e div d for every
0 <= e < 2^14 and 1 <= d <= 8192 (a block holds at most 8192 points; transform lengths are at
most 4608).  Here the same float32 arithmetic runs over that whole range, with reciprocals
anywhere within two ulps of 1/d, and a scale factor too small or too large must fail.
"""
import numpy as np

E = np.arange(1 << 14, dtype=np.int64)
EF = E.astype(np.float32)


def _mismatches(scale):
    c = np.float32(scale)
    bad = 0
    for d in range(1, 8193):
        r0 = np.float32(1.0 / d)
        for k in (-2, -1, 0, 1, 2):
            r = r0
            for _ in range(abs(k)):
                r = np.nextafter(r, np.float32(np.inf if k > 0 else 0.0), dtype=np.float32)
            rd = np.float32(r * c)
            q = (EF * rd).astype(np.int64)   # float32 product, truncated toward zero
            bad += int(np.count_nonzero(q != E // d))
    return bad


def test_rounded_up_reciprocal_division_is_exact():
    assert _mismatches(1 + 2.0 ** -16) == 0


def test_the_check_fails_without_the_margin_or_with_too_much():
    assert _mismatches(1.0) > 0          # truncation below an integer quotient
    assert _mismatches(1 + 2.0 ** -9) > 0   # excess past the next integer
