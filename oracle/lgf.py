"""Free-space lattice Green's function (LGF) of the 7-point operator, FP64, CPU.

Paper, Sec. 2.2: the LGF G_sigma solves  L G = delta  on the infinite lattice, with
L u(n) = (6 + s) u(n) - sum of the 6 neighbours (h = 1 normalisation, s = sigma h^2).
Its Fourier form (eq. "lgf") turns, through Watson's transformation (eq. "lgf_bessel",
written there for sigma = 0; the factor exp(-s t) carries sigma > 0), into

    G_s(a, b, c) = int_0^inf exp(-(6+s) t) I_a(2t) I_b(2t) I_c(2t) dt
                 = int_0^inf exp(-s t) Ĩ_a(2t) Ĩ_b(2t) Ĩ_c(2t) dt,   Ĩ_n(x) = exp(-x) I_n(x).

Following the same section, the integral is split at a large T*: a quadrature rule on
[0, T*] and, beyond T*, the large-argument asymptotic series of I_n (Abramowitz-Stegun)
integrated term by term.  The sign convention is the positive one of eq. "lgf":
G_0(0,0,0) = 0.25273..., half the Gamma-function closed form printed in Sec. 2.2.

The table stores only 0 <= a <= b <= c <= R (the 1/48 symmetry of Sec. 4); entry
(a, b, c) sits at index c(c+1)(c+2)/6 + b(b+1)/2 + a.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

U_LO = -45.0          # exp(-45) ~ 3e-20: the integrand is O(t) near t = 0
K_TAIL = 12           # terms of the asymptotic (Hankel) series kept in the tail


def table_size(R: int) -> int:
    return (R + 1) * (R + 2) * (R + 3) // 6


def sorted_index(a, b, c):
    """Index of the sorted triple a <= b <= c in the 1/48-symmetric table."""
    return c * (c + 1) * (c + 2) // 6 + b * (b + 1) // 2 + a


def canonical(d):
    """|components| sorted ascending; d has shape (..., 3), integer."""
    d = np.abs(np.asarray(d, dtype=np.int64))
    return np.sort(d, axis=-1)


def tail_start(R: int) -> float:
    """T* such that every factor's asymptotic series ratio n^2/(4T*) <= 0.05 for n <= R."""
    return 5.0 * R * R + 50.0


def hankel_coeffs(n: int, K: int = K_TAIL) -> np.ndarray:
    """alpha_k with Ĩ_n(x) ~ (2 pi x)^(-1/2) sum_k alpha_k x^(-k)  (mu = 4 n^2).

    alpha_k = (-1)^k prod_{j=1..k} (mu - (2j-1)^2) / (k! 8^k)   (Sec. 2.2, large-argument series).
    """
    mu = 4.0 * n * n
    a = np.empty(K + 1)
    a[0] = 1.0
    for k in range(1, K + 1):
        a[k] = a[k - 1] * (-(mu - (2 * k - 1) ** 2)) / (8.0 * k)
    return a


def tail_moments(s: float, T: float, kmax: int) -> np.ndarray:
    """J_k = int_T^inf exp(-s t) t^(-3/2-k) dt for k = 0..kmax.

    s = 0: T^(-1/2-k) / (k + 1/2).  s > 0: s^(k+1/2) Gamma(-k-1/2, sT), by the downward
    recurrence Gamma(a, x) = (Gamma(a+1, x) - x^a e^-x) / a from Gamma(1/2, x) = sqrt(pi) erfc(sqrt x).
    """
    J = np.empty(kmax + 1)
    if s == 0.0:
        for k in range(kmax + 1):
            p = k + 0.5
            J[k] = T ** (-p) / p
        return J
    x = s * T
    g = math.sqrt(math.pi) * math.erfc(math.sqrt(x))     # Gamma(1/2, x)
    a = 0.5
    for k in range(kmax + 1):
        # step a -> a - 1 : Gamma(a-1, x) = (Gamma(a, x) - x^(a-1) e^-x) / (a - 1)
        g = (g - x ** (a - 1.0) * math.exp(-x)) / (a - 1.0)
        a -= 1.0
        J[k] = s ** (k + 0.5) * g
    return J


def _tail_entry(n, s, T):
    """int_T^inf of the integrand via the product of three asymptotic series."""
    c = np.array([1.0])
    for m in n:
        c = np.convolve(c, hankel_coeffs(int(m)))[:K_TAIL + 1]
    J = tail_moments(s, T, K_TAIL)
    # Ĩ_n(2t) ~ (4 pi t)^(-1/2) sum_k alpha_k (2t)^(-k)
    k = np.arange(K_TAIL + 1)
    return (4.0 * math.pi) ** -1.5 * float(np.sum(c * 2.0 ** (-k) * J))


def lgf_entry(n, s: float = 0.0, R: int | None = None) -> float:
    """G_s(n) for one offset by adaptive Gauss-Kronrod quadrature (scipy QUADPACK) + tail.

    The finite part is integrated in u = ln t (dt = t du) over [U_LO, ln T*].
    """
    a, b, c = (int(v) for v in canonical(n))
    T = tail_start(max(c, 1) if R is None else R)

    def f(u):
        t = math.exp(u)
        x = 2.0 * t
        return t * math.exp(-s * t) * special.ive(a, x) * special.ive(b, x) * special.ive(c, x)

    val, _ = integrate.quad(f, U_LO, math.log(T), epsabs=1e-20, epsrel=2e-14, limit=2000)
    return val + _tail_entry((a, b, c), s, T)


def _gauss_legendre_nodes(u_hi: float, npts: int = 16):
    """Composite Gauss-Legendre nodes in u: width-4 panels on [U_LO, -6], width-1 panels above."""
    x, w = np.polynomial.legendre.leggauss(npts)
    edges = list(np.arange(U_LO, -6.0, 4.0)) + list(np.arange(-6.0, u_hi, 1.0)) + [u_hi]
    edges = sorted(set(float(e) for e in edges))
    U, W = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        U.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        W.append(0.5 * (hi - lo) * w)
    return np.concatenate(U), np.concatenate(W)


def lgf_table(R: int, s: float = 0.0) -> np.ndarray:
    """All G_s(a,b,c), 0 <= a <= b <= c <= R, in sorted-index order (FP64).

    Same split as lgf_entry, with a fixed composite Gauss-Legendre rule in u = ln t on
    [U_LO, ln T*] applied to every entry at once, and the term-by-term tail beyond T*.
    """
    R = int(R)
    T = tail_start(max(R, 1))
    U, W = _gauss_legendre_nodes(math.log(T))
    t = np.exp(U)
    X = W * t * np.exp(-s * t)                                  # quadrature weight x dt/du x e^{-st}
    B = special.ive(np.arange(R + 1)[None, :], 2.0 * t[:, None])  # Q x (R+1): Ĩ_n(2 t_q)

    # tail: sum_{i,j,l} A[a,i] A[b,j] A[c,l] J_{i+j+l},  A[n,k] = alpha_k(n) 2^-k
    K = K_TAIL
    A = np.stack([hankel_coeffs(n, K) * 2.0 ** (-np.arange(K + 1)) for n in range(R + 1)])
    J = tail_moments(s, T, 3 * K) * (4.0 * math.pi) ** -1.5
    out = np.empty(table_size(R))
    ii = np.arange(K + 1)
    for c in range(R + 1):
        Bc = B[:, : c + 1]
        M = Bc.T @ (Bc * (X * B[:, c])[:, None])                 # (c+1) x (c+1), finite part
        Jc = np.array([np.dot(A[c], J[m: m + K + 1]) for m in range(2 * K + 1)])
        H = Jc[ii[:, None] + ii[None, :]]                        # Hankel matrix in (i, j)
        Ac = A[: c + 1]
        M = M + Ac @ H @ Ac.T
        rows, cols = np.tril_indices(c + 1)                      # b = row, a = col <= b
        base = c * (c + 1) * (c + 2) // 6
        out[base + rows * (rows + 1) // 2 + cols] = M[rows, cols]
    return out


class LGFTable:
    """Dense lookup of G_s on all offsets with |component| <= R."""

    def __init__(self, R: int, s: float = 0.0, values: np.ndarray | None = None):
        self.R = int(R)
        self.s = float(s)
        self.values = lgf_table(self.R, self.s) if values is None else np.asarray(values)

    CUBE_MAX_R = 128

    def cube(self):
        """The table unfolded by its 48 symmetries onto every offset in [-R, R]^3."""
        if getattr(self, "_cube", None) is None:
            r = np.arange(-self.R, self.R + 1)
            d = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1)
            self._cube = self.lookup_sorted(d)
        return self._cube

    def lookup_sorted(self, d):
        d = canonical(d)
        if d.size and d.max() > self.R:
            raise ValueError(f"offset beyond table radius {self.R}")
        return self.values[sorted_index(d[..., 0], d[..., 1], d[..., 2])]

    def pairs(self, targets, sources):
        """Matrix G_s(m - n) for every target m (rows) and source n (columns)."""
        targets = np.asarray(targets, dtype=np.int64)
        sources = np.asarray(sources, dtype=np.int64)
        if self.R > self.CUBE_MAX_R:
            return self(targets[:, None, :] - sources[None, :, :])
        S = 2 * self.R + 1
        w = np.array([S * S, S, 1], dtype=np.int64)
        lo = np.minimum(targets.min(axis=0), sources.min(axis=0)) if len(targets) and len(sources) else 0
        hi = np.maximum(targets.max(axis=0), sources.max(axis=0)) if len(targets) and len(sources) else 0
        if np.any(np.asarray(hi) - np.asarray(lo) > self.R):
            raise ValueError(f"offset beyond table radius {self.R}")
        centre = self.R * (S * S + S + 1)
        km = targets @ w
        kn = sources @ w
        return self.cube().reshape(-1)[centre + km[:, None] - kn[None, :]]

    def __call__(self, d):
        """G_s at integer offsets d (shape (..., 3))."""
        d = np.asarray(d, dtype=np.int64)
        if self.R > self.CUBE_MAX_R:
            return self.lookup_sorted(d)
        if d.size and np.abs(d).max() > self.R:
            raise ValueError(f"offset beyond table radius {self.R}")
        R = self.R
        return self.cube()[d[..., 0] + R, d[..., 1] + R, d[..., 2] + R]

    def stencil_residual(self):
        """(6+s)G(n) - sum_6 G(n +- e_i) - delta(n) at all canonical n with c <= R-1."""
        R = self.R - 1
        idx = []
        for c in range(R + 1):
            for b in range(c + 1):
                for a in range(b + 1):
                    idx.append((a, b, c))
        n = np.array(idx, dtype=np.int64)
        res = (6.0 + self.s) * self(n)
        for e in np.eye(3, dtype=np.int64):
            res -= self(n + e) + self(n - e)
        res[0] -= 1.0
        return n, res
