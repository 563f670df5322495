"""Algorithm 1 of the paper (unfitted BAE, double-layer formulation), end to end, FP64, CPU.

  PrecomputeLGF(sigma)          -> lgf.LGFTable over every offset that occurs
  ClassifyPoints                -> geometry.build
  particular solution u_p       -> operators.volume_potential (free-space reading)
  Phi, matrix-free D            -> operators.bae_apply
  b = g - Phi u_p               -> operators.rhs
  q_d = GMRES(A, b)             -> gmres.gmres
  u_gamma = [D+ q_d ; D- q_d]   -> operators.double_layer on gamma
  u = u_p + D q_d on M+         -> operators.double_layer (+ volume_potential) on M+
Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from . import geometry, gmres, lgf, operators


def setup(problem):
    geo = geometry.from_problem(problem)
    s = problem.sigma * problem.h ** 2
    G = lgf.LGFTable(geo.max_offset(), s)
    return geo, G


def solve(problem, geo=None, G=None, rhs_index=0, tol=None, maxit=500, grid=False):
    if geo is None or G is None:
        geo, G = setup(problem)
    tol = problem.tol if tol is None else tol
    f = problem.f_grid()
    gx = problem.g(geo.xstar, rhs_index)
    b = operators.rhs(geo, G, gx, f)
    q, hist, conv = gmres.gmres(lambda x: operators.bae_apply(geo, G, x), b, tol=tol, maxit=maxit)
    T = operators.gamma_targets(geo)
    u_gamma = operators.double_layer(geo, G, q, T)
    if f is not None:
        u_gamma = u_gamma + operators.volume_potential(geo, G, f, T)
    out = dict(q=q, history=np.array(hist), converged=conv, u_gamma=u_gamma, b=b,
               true_residual=np.linalg.norm(b - operators.bae_apply(geo, G, q)) / np.linalg.norm(b))
    if grid:
        mp = geo.mplus
        u = np.full(geo.n, np.nan)
        um = operators.double_layer(geo, G, q, mp)
        if f is not None:
            um = um + operators.volume_potential(geo, G, f, mp)
        u[tuple(mp.T)] = um
        u[tuple(T.T)] = u_gamma
        out["u_grid"] = u
    return out
