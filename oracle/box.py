"""The particular solution on the finite grid (Algorithm 1, first step): u_p = G_h[chi_{M+} f].

G_h inverts the 7-point operator (L_h u)(m) = (6 + s) u(m) - sum of the six neighbours of m on
the interior nodes of the box, with u = 0 on the box's boundary nodes (Sec. 2.1, the finite
auxiliary domain; the paper solves it by FFT).  Here the sine transform of type I, which
diagonalises L_h on that box, is the library step (scipy.fft.dstn, orthonormal); the
eigenvalue of the sine mode k is (6 + s) - 2 sum_d cos(pi k_d / (N_d + 1)).

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def particular_box(geo, s, f_grid):
    """u_p on the whole grid (zero on the box boundary) for the source h^2 chi_{M+} f."""
    n = tuple(int(v) for v in geo.n)
    q = np.zeros(n)
    mp = geo.mplus
    q[tuple(mp.T)] = geo.h ** 2 * np.asarray(f_grid, dtype=float).reshape(n)[tuple(mp.T)]
    inner = q[1:-1, 1:-1, 1:-1]
    N = inner.shape
    lam = (6.0 + s) * np.ones(N)
    for d in range(3):
        k = np.arange(1, N[d] + 1)
        shape = [1, 1, 1]
        shape[d] = N[d]
        lam = lam - 2.0 * np.cos(np.pi * k / (N[d] + 1)).reshape(shape)
    uh = sfft.dstn(inner, type=1, norm="ortho") / lam
    u = np.zeros(n)
    u[1:-1, 1:-1, 1:-1] = sfft.idstn(uh, type=1, norm="ortho")
    return u
