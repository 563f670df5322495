"""The direct formulation of the boundary algebraic equations, FP64, CPU.

Paper, Sec. 3.1: the lattice form of Green's second identity (Duffin) over E = M+, applied to a
grid function u with L u = 0 on M+ and to the free-space LGF peaked at a point p* of M+,
gives Green's third identity on the lattice.  With L = (6+s) I - (sum of the six shifts) and
the positive G of this oracle (L G = delta), it reads
    u(p*) = sum over edges (p, q) of [ G(p - p*) u(q) - G(q - p*) u(p) ],
the edges being the neighbour pairs with p in M+ and q outside M+, i.e. p in gamma+ and
q in gamma- (eq. "direct_bae").  For p* in gamma+ this is the boundary algebraic equation
(I - P+) v_{gamma+} = P- v_{gamma-} of eq. "beq_bae" with
    (P+ v+)(p*) = - sum_edges G(q - p*) v+(p)     ("G_{gamma-}", reduced from gamma- to gamma+)
    (P- v-)(p*) =   sum_edges G(p - p*) v-(q)     ("G_{gamma+}", extended from gamma+ to gamma-)
(the paper prints P+ := G_{gamma-}, P- := -G_{gamma+} in its negative sign convention).  The
system (eq. "direct_sys") closes it with the Dirichlet rows of Sec. 2.1:
    (I - P+) v+ - P- v- = 0        on gamma+
    Phi+ v+ + Phi- v-   = b        on gamma-,   b = g - Phi u_p.
The unknowns are v on gamma itself, in the order [gamma+ ; gamma-]; u_gamma = v + u_p and,
by the same identity, u(m) = u_p(m) + sum_edges [G(p - m) v(q) - G(q - m) v(p)] on M+.

Everything is evaluated literally, one G per (target, edge endpoint).
Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from . import gmres, operators
from .geometry import DIRS

BLOCK = 64


def boundary_edges(geo):
    """The neighbour pairs (p, q), p in gamma+, q in gamma-, as index pairs into gamma_plus and
    gamma_minus, in lexicographic order of q then direction."""
    n = tuple(int(v) for v in geo.n)
    pos = -np.ones(n, dtype=np.int64)
    pos[tuple(geo.gamma_plus.T)] = np.arange(len(geo.gamma_plus))
    out = []
    for qi, q in enumerate(geo.gamma_minus):
        for d in DIRS:
            m = q + d
            if np.all(m >= 0) and np.all(m < np.asarray(n)) and geo.inside[tuple(m)]:
                out.append((pos[tuple(m)], qi))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def representation(geo, G, v, targets, edges=None):
    """sum_edges [ G(p - m) v(q) - G(q - m) v(p) ] at m in targets, v on gamma ([gamma+; gamma-])."""
    targets = np.asarray(targets, dtype=np.int64)
    edges = boundary_edges(geo) if edges is None else edges
    npl = len(geo.gamma_plus)
    P = geo.gamma_plus[edges[:, 0]]
    Q = geo.gamma_minus[edges[:, 1]]
    vp = v[edges[:, 0]]
    vq = v[npl + edges[:, 1]]
    out = np.empty(len(targets))
    for b0 in range(0, len(targets), BLOCK):
        m = targets[b0:b0 + BLOCK]
        out[b0:b0 + BLOCK] = (G.pairs(m, P) * vq[None] - G.pairs(m, Q) * vp[None]).sum(axis=1)
    return out


def direct_apply(geo, G, v, edges=None):
    """The direct system's operator: [ v+ - (representation at gamma+) ; Phi+ v+ + Phi- v- ]."""
    npl = len(geo.gamma_plus)
    top = v[:npl] - representation(geo, G, v, geo.gamma_plus, edges)
    return np.concatenate([top, operators.closure(geo, v)])


def dense_p(geo, G):
    """Dense P+ (|gamma+| x |gamma+|) and P- (|gamma+| x |gamma-|), tiny grids only."""
    edges = boundary_edges(geo)
    Pp = np.zeros((len(geo.gamma_plus), len(geo.gamma_plus)))
    Pm = np.zeros((len(geo.gamma_plus), len(geo.gamma_minus)))
    for pi, qi in edges:
        Pp[:, pi] -= G.pairs(geo.gamma_plus, geo.gamma_minus[qi][None])[:, 0]
        Pm[:, qi] += G.pairs(geo.gamma_plus, geo.gamma_plus[pi][None])[:, 0]
    return Pp, Pm


def solve(problem, geo, G, tol=1e-12, maxit=1000, rhs_index=0, grid=False):
    """GMRES on the direct system; returns v, u_gamma (= v + u_p) and the history."""
    f = problem.f_grid()
    gx = problem.g(geo.xstar, rhs_index)
    b = operators.rhs(geo, G, gx, f)
    npl = len(geo.gamma_plus)
    bb = np.concatenate([np.zeros(npl), b])
    edges = boundary_edges(geo)
    v, hist, conv = gmres.gmres(lambda x: direct_apply(geo, G, x, edges), bb, tol=tol, maxit=maxit)
    T = operators.gamma_targets(geo)
    u_gamma = v.copy()
    if f is not None:
        u_gamma = u_gamma + operators.volume_potential(geo, G, f, T)
    out = dict(v=v, u_gamma=u_gamma, history=np.array(hist), converged=conv, b=bb)
    if grid:
        mp = geo.mplus
        um = representation(geo, G, v, mp, edges)
        if f is not None:
            um = um + operators.volume_potential(geo, G, f, mp)
        u = np.full(geo.n, np.nan)
        u[tuple(mp.T)] = um
        u[tuple(geo.gamma_minus.T)] = u_gamma[npl:]
        out["u_grid"] = u
    return out
