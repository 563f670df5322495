"""Pins of the oracle's lattice Green's function (Sec. 2.2 of the paper) to values and
identities fixed independently of it."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import lgf


def mp_lgf(n, s=0.0, dps=35):
    """G_s(n) by mpmath's tanh-sinh quadrature of the Bessel integral at `dps` digits."""
    with mp.workdps(dps):
        a, b, c = n
        s = mp.mpf(s)
        f = lambda t: mp.exp(-(6 + s) * t) * mp.besseli(a, 2 * t) * mp.besseli(b, 2 * t) * mp.besseli(c, 2 * t)
        return float(mp.quad(f, [0, 1, 10, 100, 1000, 10000, mp.inf]))


def test_watson_closed_forms():
    # Sec. 2.2 prints two Gamma-function closed forms for the sigma = 0 value at the origin;
    # both equal Watson's integral (1/pi^3) int dθ / (3 - sum cos), which is twice G_0(0)
    # in the normalisation of eq. "lgf" (denominator 6 - 2 sum cos).
    with mp.workdps(30):
        g1 = mp.sqrt(6) / (96 * mp.pi ** 3) * mp.gamma(mp.mpf(1) / 24) * mp.gamma(mp.mpf(5) / 24) \
            * mp.gamma(mp.mpf(7) / 24) * mp.gamma(mp.mpf(11) / 24)
        g2 = (mp.sqrt(3) - 1) / (96 * mp.pi ** 3) * (mp.gamma(mp.mpf(1) / 24) * mp.gamma(mp.mpf(11) / 24)) ** 2
        assert abs(g1 - g2) < mp.mpf(10) ** -25
        half = float(g1 / 2)
    t = lgf.LGFTable(4, 0.0)
    assert abs(t(np.array([0, 0, 0])) - half) < 2e-16
    assert abs(lgf.lgf_entry((0, 0, 0), 0.0) - half) < 2e-16


@pytest.mark.parametrize("s", [0.0, 1.526e-4, 0.05, 2.0])
def test_first_shell_from_the_stencil(s):
    # L G = delta at the origin with the 6 equal neighbours: (6+s) G(0) - 6 G(e1) = 1.
    t = lgf.LGFTable(3, s)
    g0, g1 = t(np.array([0, 0, 0])), t(np.array([1, 0, 0]))
    assert abs(g1 - ((6.0 + s) * g0 - 1.0) / 6.0) < 2e-16


@pytest.mark.parametrize("s", [0.0, 1.526e-4, 0.0488, 2.0])
def test_stencil_residual_everywhere(s):
    # eq. "lgf_delta": (6+s) G(n) - sum_6 G(n +- e_i) = delta(n) on the whole table.
    t = lgf.LGFTable(40, s)
    n, res = t.stencil_residual()
    assert np.abs(res).max() < 2e-15


@pytest.mark.parametrize("n,s", [((1, 1, 0), 0.0), ((2, 0, 0), 0.0), ((3, 2, 1), 0.0),
                                 ((20, 5, 3), 0.0), ((0, 0, 0), 0.0488), ((4, 1, 0), 0.0488),
                                 ((30, 0, 0), 1e-4)])
def test_against_mpmath(n, s):
    ref = mp_lgf(n, s)
    t = lgf.LGFTable(max(n) + 1, s)
    assert abs(t(np.array(n)) - ref) <= 1e-14 * ref
    assert abs(lgf.lgf_entry(n, s) - ref) <= 1e-13 * ref


def test_table_matches_adaptive_quadrature():
    # the vectorised fixed rule against QUADPACK's adaptive Gauss-Kronrod (paper: "adaptive
    # Gauss Kronrod method" is an alternative evaluation of eq. "lgf_bessel")
    rng = np.random.default_rng(7)
    for s in (0.0, 6.1e-4):
        t = lgf.LGFTable(117, s)
        for _ in range(12):
            n = np.sort(rng.integers(0, 118, 3))
            e = lgf.lgf_entry(tuple(n), s, R=117)
            assert abs(t(n) - e) <= 2e-14 * e


def q3_expansion(n, c=-228):
    """Sec. 2.2's q = 3 expansion of G_0 in the positive sign convention, written out in the
    offset components (c: the coefficient printed as -288, read as -228)."""
    j, k, l = (float(v) for v in n)
    r = math.sqrt(j * j + k * k + l * l)
    P4 = j ** 4 + k ** 4 + l ** 4 - 3 * (j * j * k * k + j * j * l * l + k * k * l * l)
    P8 = (c * (k * k * l * l * j ** 4 + k * k * l ** 4 * j * j + k ** 4 * l * l * j * j)
          + 621 * (j ** 4 * k ** 4 + l ** 4 * k ** 4 + j ** 4 * l ** 4)
          - 244 * (k * k * j ** 6 + l * l * j ** 6 + k ** 6 * j * j + l ** 6 * j * j + k * k * l ** 6 + k ** 6 * l * l)
          + 23 * (j ** 8 + k ** 8 + l ** 8))
    return 1 / (4 * math.pi * r) + P4 / (16 * math.pi * r ** 7) + P8 / (128 * math.pi * r ** 13)


def test_far_field_decay_and_the_A3_reading():
    # Sec. 2.2: G_0(n) -> 1/(4 pi |n|) as |n| -> inf, with the q-term expansion error
    # O(|n|^(-2q-1)).  In the positive sign convention of eq. "lgf" the q=3 expansion only
    # decays like |n|^-6 relative if the coefficient printed as -288 reads -228 (the
    # symmetric-polynomial form 23p^4 - 336p^2e2 + 1155e2^2 - 1134p e3 of the bracket).
    t = lgf.LGFTable(120, 0.0)
    A3 = q3_expansion
    r = 117.0
    assert abs(4 * math.pi * r * t(np.array([117, 0, 0])) - 1.0) < 2e-5
    e1 = [abs(A3(n, -228) / t(np.array(n)) - 1) for n in ((20, 20, 5), (40, 40, 10), (80, 80, 20))]
    e2 = [abs(A3(n, -288) / t(np.array(n)) - 1) for n in ((20, 20, 5), (40, 40, 10), (80, 80, 20))]
    assert 40 < e1[0] / e1[1] < 100 and 40 < e1[1] / e1[2] < 100      # ~2^6
    assert 10 < e2[0] / e2[1] < 25 and 10 < e2[1] / e2[2] < 25         # ~2^4
    assert e1[1] < 5e-11


def test_single_entries_at_the_largest_offsets():
    # Lattice coordinates reach 2048 (2049 nodes per axis).  That far out the q = 3 expansion
    # leaves a relative error of order |n|^-6 (below 1e-19), so it fixes G_0 to rounding, and
    # the oracle's single-entry quadrature with its analytic tail must agree.
    for n in ((2048, 0, 0), (2000, 3, 1), (1500, 700, 2), (1024, 1024, 1024), (2048, 2048, 2048), (300, 5, 0)):
        v = lgf.lgf_entry(np.array(n), 0.0)
        assert abs(q3_expansion(n) / v - 1) < 1e-12, (n, q3_expansion(n) / v - 1)


def test_small_sigma_limit():
    # For small s the modified-Helmholtz LGF at the origin behaves like the continuous
    # Yukawa kernel's regular part: G_s(0) = G_0(0) - sqrt(s)/(4 pi) + O(s).
    g0 = lgf.LGFTable(2, 0.0)(np.array([0, 0, 0]))
    for s in (1e-6, 1e-8):
        gs = lgf.LGFTable(2, s)(np.array([0, 0, 0]))
        assert abs(gs - g0 + math.sqrt(s) / (4 * math.pi)) < 3 * s


def test_yukawa_far_field_form():
    # sigma > 0: the Fourier-symbol expansion of 1/(s + 6 - 2 sum cos) with the Yukawa
    # functions g_k gives G_s(n) ~ e^(-u)/(4 pi |n|) [1 + T2], u = sqrt(s)|n|,
    # T2 |n|^2 = (1 + u)(1 - 5x)/4 - u^2 x/2 + u^3 (1 - 2x)/24, x = e2/|n|^4.  Against the
    # table: the dropped term is O(|n|^-4) at fixed u (error ratio ~2^4 when |n| doubles
    # along a ray), and at s = 0 it is the paper's q = 2 form.
    # The device evaluates the exponentiated form e^(-u + T2) / (4 pi |n|), which differs from
    # the expansion by T2^2 / 2 = O(|n|^-4), the order of the dropped term: both are pinned.
    def form(n, s, exponent=False):
        j, k, l = (float(v) for v in n)
        X, Y, Z = j * j, k * k, l * l
        r2 = X + Y + Z
        r = math.sqrt(r2)
        x = (X * Y + Y * Z + Z * X) / r2 ** 2
        u = math.sqrt(s) * r
        T2 = ((1 + u) * (1 - 5 * x) / 4 - u * u * x / 2 + u ** 3 * (1 - 2 * x) / 24) / r2
        return math.exp(-u) / (4 * math.pi * r) * (math.exp(T2) if exponent else 1 + T2)

    s = 1.5e-4                                          # kappa^2 h^2 of the 257^3 star
    t = lgf.LGFTable(150, s)
    rays = [(1, 0, 0), (1, 1, 0)]                      # directions where the dropped term is largest
    for exponent in (False, True):
        for d in rays:
            errs = []
            for m in (12, 24, 48):
                n = np.array([m * c for c in d])
                errs.append(abs(form(n, s, exponent) / t(n) - 1))
            assert 8 < errs[0] / errs[1] < 32 and 8 < errs[1] / errs[2] < 32, errs
        n = np.array([56, 0, 0])
        assert abs(form(n, s, exponent) / t(n) - 1) < 1.5e-7   # the worst offset beyond the LDS radius
    t0 = lgf.LGFTable(60, 0.0)
    n = np.array([40, 25, 10])
    r = math.sqrt(40 ** 2 + 25 ** 2 + 10 ** 2)
    x = (40 ** 2 * 25 ** 2 + 25 ** 2 * 10 ** 2 + 10 ** 2 * 40 ** 2) / r ** 4
    q2 = 1 / (4 * math.pi * r) * (1 + (1 - 5 * x) / (4 * r * r))
    assert abs(form(n, 0.0) - q2) < 1e-15 * q2 and abs(q2 / t0(n) - 1) < 1e-6


def test_the_257_star_table():
    # The table the 257^3 modified-Helmholtz parity cases read (kappa^2 = 10, h = 1/256,
    # offsets to 238): the stencil identity on every entry, QUADPACK's adaptive rule at
    # large offsets and mpmath at one off-axis offset.
    s = 10.0 / 256 ** 2
    t = lgf.LGFTable(238, s)
    _, res = t.stencil_residual()
    assert np.abs(res).max() < 2e-15
    for n in [(237, 0, 0), (200, 150, 3), (120, 120, 120), (238, 238, 238), (61, 17, 5), (238, 1, 0)]:
        e = lgf.lgf_entry(n, s, R=238)
        assert abs(t(np.array(n)) - e) <= 1e-13 * e, n
    ref = mp_lgf((90, 40, 7), s, dps=20)
    assert abs(t(np.array((90, 40, 7))) - ref) <= 1e-13 * ref
