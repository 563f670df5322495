"""Unrestarted GMRES, FP64, CPU (Saad & Schultz), as used in Sec. 4 of the paper:
"vanilla" GMRES, no preconditioner, zero initial guess, stopped on the relative residual.

Arnoldi by modified Gram-Schmidt, the Hessenberg least-squares problem by Givens rotations;
the residual estimate after step k is |g_{k+1}| / ||b||.
Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def gmres(apply, b, tol=1e-10, maxit=500):
    """Solve A x = b; returns (x, history, converged). history[k] = estimate after k+1 steps."""
    b = np.asarray(b, dtype=float)
    n = len(b)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n), [], True
    m = min(maxit, n)
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[0] = b / beta
    hist = []
    k_done = 0
    converged = False
    for k in range(m):
        w = apply(V[k])
        for i in range(k + 1):                       # modified Gram-Schmidt
            H[i, k] = np.dot(V[i], w)
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] != 0.0:
            V[k + 1] = w / H[k + 1, k]
        for i in range(k):                           # previous rotations on the new column
            a, c = H[i, k], H[i + 1, k]
            H[i, k] = cs[i] * a + sn[i] * c
            H[i + 1, k] = -sn[i] * a + cs[i] * c
        a, c = H[k, k], H[k + 1, k]                  # new rotation zeroing H[k+1, k]
        r = np.hypot(a, c)
        cs[k], sn[k] = a / r, c / r
        H[k, k] = r
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / beta)
        k_done = k + 1
        if hist[-1] <= tol or H[k, k] == 0.0:
            converged = hist[-1] <= tol
            break
    y = np.zeros(k_done)
    for i in range(k_done - 1, -1, -1):              # back substitution R y = g
        y[i] = (g[i] - np.dot(H[i, i + 1:k_done], y[i + 1:])) / H[i, i]
    x = V[:k_done].T @ y
    return x, hist, converged
