"""Layer potentials and the boundary algebraic operator, FP64, CPU.

Paper, Sec. 3.2:
  single layer kernel   S(m, n) = G_s(m - n)
  double layer kernel   D(m, n) = sum_{k in D_n} [ G_s(m - n) - G_s(m - k) ],  n in gamma-
  double layer potential v_m = sum_{n in gamma-} D(m, n) q_d(n)
(The kernel argument is the componentwise offset vector; G_s is 48-fold symmetric.)
Sec. 3.4, eq. "double_bae": the boundary algebraic system (Phi+ D+ + Phi- D-) q_d = b,
with D+- the rows of D at gamma+- and Phi+- the Dirichlet-closure rows of Sec. 2.1.
Algorithm 1: u_gamma = [D+ q_d ; D- q_d].  Sec. 2.1 eq. "discrete_green" / Algorithm 1:
u = u_p + (double layer potential) on M+, u_p = G_h[chi_{M+} f] (here the free-space
volume potential h^2 sum_{n in M+} G_s(m - n) f(n), the unbounded-domain reading of Sec. 3.5).

Everything is evaluated literally: one G per (target, n) plus one per (target, n, k).
Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

BLOCK = 64


def gamma_targets(geo):
    """The targets T = gamma in output order: gamma+ (lexicographic) then gamma- (lexicographic)."""
    return np.concatenate([geo.gamma_plus, geo.gamma_minus])


def double_layer(geo, G, q, targets):
    """v(m) = sum_{n in gamma-} q(n) sum_{k in D_n} [G(m - n) - G(m - k)]  for m in targets."""
    targets = np.asarray(targets, dtype=np.int64)
    q = np.asarray(q, dtype=float)
    en = geo.gamma_minus[geo.edges[:, 0]]          # source node n of each (n, k) pair
    ek = geo.ext[geo.edges[:, 1]]                  # its outside neighbour k
    qe = q[geo.edges[:, 0]]
    v = np.empty(len(targets))
    for b0 in range(0, len(targets), BLOCK):
        m = targets[b0:b0 + BLOCK]
        v[b0:b0 + BLOCK] = ((G.pairs(m, en) - G.pairs(m, ek)) * qe[None]).sum(axis=1)
    return v


def single_layer(geo, G, q, targets):
    """v(m) = sum_{n in gamma-} G(m - n) q(n)."""
    targets = np.asarray(targets, dtype=np.int64)
    v = np.empty(len(targets))
    for b0 in range(0, len(targets), BLOCK):
        m = targets[b0:b0 + BLOCK]
        v[b0:b0 + BLOCK] = (G.pairs(m, geo.gamma_minus) * q[None]).sum(axis=1)
    return v


def closure(geo, v_gamma):
    """Phi+ v_{gamma+} + Phi- v_{gamma-}: row q reads (1 - t_q) v(q) + t_q v(p_q)."""
    npl = len(geo.gamma_plus)
    v_minus = v_gamma[npl:]
    v_plus = v_gamma[:npl]
    return (1.0 - geo.t) * v_minus + geo.t * v_plus[geo.partner]


def bae_apply(geo, G, q):
    """A q = (Phi+ D+ + Phi- D-) q."""
    return closure(geo, double_layer(geo, G, q, gamma_targets(geo)))


def dense_double_layer(geo, G, targets):
    """Matrix D(m, n), m in targets, n in gamma-  (tiny grids only)."""
    targets = np.asarray(targets, dtype=np.int64)
    D = np.zeros((len(targets), len(geo.gamma_minus)))
    for (ni, ki) in geo.edges:
        n = geo.gamma_minus[ni]
        k = geo.ext[ki]
        D[:, ni] += G.pairs(targets, n[None])[:, 0] - G.pairs(targets, k[None])[:, 0]
    return D


def dense_single_layer(geo, G, targets):
    targets = np.asarray(targets, dtype=np.int64)
    return G.pairs(targets, geo.gamma_minus)


def dense_operator(geo, G):
    D = dense_double_layer(geo, G, gamma_targets(geo))
    npl = len(geo.gamma_plus)
    Dp, Dm = D[:npl], D[npl:]
    return (1.0 - geo.t)[:, None] * Dm + geo.t[:, None] * Dp[geo.partner]


def volume_potential(geo, G, f_grid, targets):
    """u_p(m) = h^2 sum_{n in M+} G(m - n) f(n)."""
    targets = np.asarray(targets, dtype=np.int64)
    src = geo.mplus
    fv = np.asarray(f_grid, dtype=float).reshape(geo.n)[tuple(src.T)]
    out = np.empty(len(targets))
    blk = max(1, BLOCK * 4096 // max(len(src), 1))
    for b0 in range(0, len(targets), blk):
        m = targets[b0:b0 + blk]
        out[b0:b0 + blk] = (G.pairs(m, src) * fv[None]).sum(axis=1)
    return geo.h ** 2 * out


def rhs(geo, G, g_xstar, f_grid=None):
    """b = g(x*) - Phi [u_p]_gamma   (Sec. 3.4; u_p = 0 when f = 0)."""
    b = np.asarray(g_xstar, dtype=float).copy()
    if f_grid is not None:
        up = volume_potential(geo, G, f_grid, gamma_targets(geo))
        b -= closure(geo, up)
    return b
