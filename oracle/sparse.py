"""The plain sparse discrete Dirichlet problem the BAE solution equals, FP64, CPU.

Paper, Sec. 2.2 (equivalence of the finite and free-space boundary equations) and
Sec. 3.2 (eq. "equal"): whatever representation is used, the density reproduces the
unique grid function u on N+ = M+ u gamma- with
    (6 + s) u(m) - sum_6 u(m +- e) = h^2 f(m)      for m in M+      (eq. "discrete", scaled by h^2)
    (1 - t_q) u(q) + t_q u(p_q)     = g(x*_q)       for q in gamma-  (eq. "bc", hat functions)
This module assembles that system and solves it with SciPy's sparse LU.
Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import DIRS


def solve(geo, s, g_xstar, f_grid=None):
    """Returns u on N+ as a full grid array (NaN outside N+)."""
    n = geo.n
    mp = geo.mplus
    gm = geo.gamma_minus
    nodes = np.concatenate([mp, gm])
    lin = np.ravel_multi_index(tuple(nodes.T), n)
    pos = -np.ones(int(np.prod(n)), dtype=np.int64)
    pos[lin] = np.arange(len(nodes))
    rows, cols, vals = [], [], []
    nm = len(mp)
    r = np.arange(nm)
    rows.append(r); cols.append(r); vals.append(np.full(nm, 6.0 + s))
    for d in DIRS:
        nb = np.ravel_multi_index(tuple((mp + d).T), n)
        rows.append(r); cols.append(pos[nb]); vals.append(np.full(nm, -1.0))
    rq = nm + np.arange(len(gm))
    pl = np.ravel_multi_index(tuple(geo.gamma_plus[geo.partner].T), n)
    rows.append(rq); cols.append(rq); vals.append(1.0 - geo.t)
    rows.append(rq); cols.append(pos[pl]); vals.append(geo.t)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(nodes), len(nodes)))
    rhs = np.zeros(len(nodes))
    if f_grid is not None:
        rhs[:nm] = geo.h ** 2 * np.asarray(f_grid, dtype=float).reshape(n)[tuple(mp.T)]
    rhs[nm:] = g_xstar
    if np.any(cols[1] < 0):
        raise ValueError("stencil leaves N+")
    u = spla.spsolve(A.tocsc(), rhs)
    out = np.full(n, np.nan)
    out[tuple(nodes.T)] = u
    return out
