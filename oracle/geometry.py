"""Point sets of the unfitted method and the Dirichlet closure, FP64, CPU.

Paper, Sec. 2.1: grid points M0 of the box, M+ = points inside Omega (level set < 0,
the convention of Sec. 4.2), M- = M0 minus M+, N+- = 7-point stencil closures of M+-,
gamma = N+ cap N-, gamma+ = gamma cap M+, gamma- = gamma cap M-.  Equivalently
gamma+ = {m in M+ with a 6-neighbour in M-} and gamma- = {q in M- with a 6-neighbour in M+};
N+ = M+ u gamma-.

Sec. 3.2 (double layer kernel): D_n = the neighbours of source node n (in gamma-) that lie
outside N+.  E = union of all D_n (the extra source nodes of the double layer).

Sec. 2.1, eq. "bc" (Dirichlet closure with hat functions): one boundary point x* per
gamma- node q, on the grid edge from q to a 6-neighbour p in M+, where the level set
vanishes; on that edge the 3-D hat functions reduce to linear interpolation, so the
closure row reads (1 - t) u(q) + t u(p) = g(x*), x* = x_q + t (x_p - x_q).
Readings (paper silent): D_n may be empty (see build); the neighbour p with the smallest t is used, ties broken in the
direction order -x, +x, -y, +y, -z, +z; t is found by bisection on the analytic level
set (60 halvings, keeping the phi >= 0 end), or by linear interpolation of node values
for a sampled level set.  A node with phi == 0 belongs to M-.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

DIRS = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], dtype=np.int64)


class GeometryError(ValueError):
    pass


def level_set(kind, center, params, X):
    """phi(X) for the analytic kinds; X has shape (..., 3).  Interior: phi < 0."""
    c = np.asarray(center, dtype=float)
    d = np.asarray(X, dtype=float) - c
    dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
    p = params
    if kind == "sphere":
        return dx * dx + dy * dy + dz * dz - p[0] * p[0]
    if kind == "ellipsoid":
        return (dx / p[0]) ** 2 + (dy / p[1]) ** 2 + (dz / p[2]) ** 2 - 1.0
    if kind == "torus":
        return (np.sqrt(dx * dx + dy * dy) - p[0]) ** 2 + dz * dz - p[1] * p[1]
    if kind == "star":
        rho = np.sqrt(dx * dx + dy * dy + dz * dz)
        theta = np.arctan2(np.sqrt(dx * dx + dy * dy), dz)
        az = np.arctan2(dy, dx)
        return rho - p[0] * (1.0 + p[1] * np.sin(p[2] * theta) * np.cos(p[3] * az))
    raise ValueError(f"unknown level-set kind {kind}")


@dataclass
class Geometry:
    n: tuple
    h: float
    origin: np.ndarray
    inside: np.ndarray          # bool (n0, n1, n2): M+
    gamma_plus: np.ndarray      # (|gamma+|, 3) int, lexicographic
    gamma_minus: np.ndarray     # (|gamma-|, 3) int, lexicographic
    ext: np.ndarray             # (|E|, 3) int, lexicographic
    edges: np.ndarray           # (n_edges, 2): (index into gamma_minus, index into ext), n in gamma-, k in D_n
    partner: np.ndarray         # (|gamma-|,) index into gamma_plus of the edge partner p
    t: np.ndarray               # (|gamma-|,) closure weight t in [0, 1)
    xstar: np.ndarray           # (|gamma-|, 3) boundary points

    @property
    def mplus(self):
        return np.argwhere(self.inside)

    def coords(self, ijk):
        return self.origin + self.h * np.asarray(ijk, dtype=float)

    def d_count(self):
        return np.bincount(self.edges[:, 0], minlength=len(self.gamma_minus))

    def max_offset(self):
        """Largest |component| of an offset between any two of N+ u E (the table radius)."""
        pts = np.concatenate([self.mplus, self.gamma_minus, self.ext])
        return int((pts.max(axis=0) - pts.min(axis=0)).max())


def _shift(mask, d):
    """out[i] = mask[i + d] (False outside the grid)."""
    out = np.zeros_like(mask)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    for ax in range(3):
        if d[ax] > 0:
            src[ax] = slice(d[ax], None)
            dst[ax] = slice(None, -d[ax])
        elif d[ax] < 0:
            src[ax] = slice(None, d[ax])
            dst[ax] = slice(-d[ax], None)
    out[tuple(dst)] = mask[tuple(src)]
    return out


def build(n, h, origin, kind, center=None, params=None, phi_nodes=None) -> Geometry:
    n = tuple(int(v) for v in n)
    origin = np.asarray(origin, dtype=float)
    ii = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), axis=-1)
    X = origin + h * ii
    if kind == "sampled":
        phi = np.asarray(phi_nodes, dtype=float).reshape(n)
    else:
        phi = level_set(kind, center, params, X)
    if not np.all(np.isfinite(phi)):
        raise GeometryError("non-finite level-set value")
    inside = phi < 0.0
    if not inside.any():
        raise GeometryError("empty interior M+")
    mp = np.argwhere(inside)
    if mp.min() < 2 or np.any(mp.max(axis=0) > np.array(n) - 3):
        raise GeometryError("interior within two nodes of the grid edge")

    nb_in = np.zeros_like(inside)
    nb_out = np.zeros_like(inside)
    for d in DIRS:
        s = _shift(inside, d)
        nb_in |= s
        nb_out |= _shift(~inside, d)
    # (nodes beyond the grid would count as M-; M+ keeps >= 2 nodes from the edge, so none is needed)
    gm_mask = (~inside) & nb_in
    gp_mask = inside & nb_out
    nplus = inside | gm_mask

    gamma_plus = np.argwhere(gp_mask)
    gamma_minus = np.argwhere(gm_mask)

    # D_n for n in gamma-: neighbours outside N+
    ext_list = []
    edge_q = []
    for qi, q in enumerate(gamma_minus):
        for d in DIRS:
            k = q + d
            if not nplus[tuple(k)]:
                ext_list.append(tuple(k))
                edge_q.append(qi)
    if len(edge_q) == 0:
        raise GeometryError("no exterior nodes")
    ext = np.array(sorted(set(ext_list)), dtype=np.int64)
    ext_lin = {tuple(v): i for i, v in enumerate(ext)}
    edges = np.array([(qi, ext_lin[k]) for qi, k in zip(edge_q, ext_list)], dtype=np.int64)
    # A gamma- node whose six neighbours all lie in N+ has an empty D_n: its double-layer
    # column is zero and its density is free.  The system stays consistent (the discrete
    # problem it is equivalent to is still uniquely solvable), so this is allowed.

    # Dirichlet closure: crossing t on every edge q -> p (p in M+), all edges at once
    gp_lin = {tuple(v): i for i, v in enumerate(gamma_plus)}
    cand_q, cand_d = [], []
    for qi, q in enumerate(gamma_minus):
        for di, d in enumerate(DIRS):
            if inside[tuple(q + d)]:
                cand_q.append(qi)
                cand_d.append(di)
    cand_q = np.array(cand_q)
    cand_d = np.array(cand_d)
    qv = gamma_minus[cand_q]
    pv = qv + DIRS[cand_d]
    xq = origin + h * qv
    xp = origin + h * pv
    if kind == "sampled":
        fq = phi[tuple(qv.T)]
        fp = phi[tuple(pv.T)]
        tc = fq / (fq - fp)
    else:
        lo = np.zeros(len(cand_q))
        hi = np.ones(len(cand_q))
        for _ in range(60):                       # bisection, keeping the phi >= 0 end at lo
            mid = 0.5 * (lo + hi)
            neg = level_set(kind, center, params, xq + mid[:, None] * (xp - xq)) < 0.0
            hi = np.where(neg, mid, hi)
            lo = np.where(neg, lo, mid)
        tc = lo
    partner = np.empty(len(gamma_minus), dtype=np.int64)
    tq = np.full(len(gamma_minus), np.inf)
    xs = np.empty((len(gamma_minus), 3))
    for c in range(len(cand_q)):                  # candidates are in direction order per q
        qi = cand_q[c]
        if tc[c] < tq[qi]:
            tq[qi] = tc[c]
            partner[qi] = gp_lin[tuple(pv[c])]
            xs[qi] = xq[c] + tc[c] * (xp[c] - xq[c])
    return Geometry(n, float(h), origin, inside, gamma_plus, gamma_minus, ext, edges, partner, tq, xs)


def from_problem(p) -> Geometry:
    return build(p.n, p.h, p.origin, p.kind, p.center, p.params)
