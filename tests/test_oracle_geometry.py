"""Pins of the oracle's point sets and Dirichlet closure (Sec. 2.1 of the paper)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry


def lattice_points_in_ball(n, h, c, r):
    """Count nodes i h with |x - c| < r column by column, from the closed form of the
    k-range of each (i, j) column (independent of the oracle's classification)."""
    count = 0
    for i in range(n):
        for j in range(n):
            rem = r * r - (i * h - c) ** 2 - (j * h - c) ** 2
            if rem <= 0:
                continue
            w = math.sqrt(rem)
            # k h in (c - w, c + w), strictly
            lo = math.floor((c - w) / h) + 1
            hi = math.ceil((c + w) / h) - 1
            lo, hi = max(lo, 0), min(hi, n - 1)
            count += max(0, hi - lo + 1)
    return count


def test_sphere_interior_count():
    p = W.laplace_sphere()
    g = geometry.from_problem(p)
    assert g.inside.sum() == lattice_points_in_ball(33, 1 / 32, 0.5, 0.4)


def test_sets_satisfy_their_definitions():
    p = W.poisson_ellipsoid(21)
    g = geometry.from_problem(p)
    inside = g.inside
    nplus = inside.copy()
    nplus[tuple(g.gamma_minus.T)] = True
    for m in g.gamma_plus:
        assert inside[tuple(m)] and any(not inside[tuple(m + d)] for d in geometry.DIRS)
    for q in g.gamma_minus:
        assert not inside[tuple(q)] and any(inside[tuple(q + d)] for d in geometry.DIRS)
    # every M+ node with an M- neighbour is in gamma+, and vice versa
    assert len(g.gamma_plus) == sum(1 for m in np.argwhere(inside)
                                    if any(not inside[tuple(m + d)] for d in geometry.DIRS))
    for (qi, ki) in g.edges:
        q, k = g.gamma_minus[qi], g.ext[ki]
        assert np.abs(q - k).sum() == 1 and not nplus[tuple(k)]
    # E is exactly the union of the D_n
    assert len(np.unique(g.edges[:, 1])) == len(g.ext)


def test_boundary_points_on_the_sphere():
    # x* = x_q + t (x_p - x_q) must solve |x* - c| = r; check t against the closed-form root
    # of the quadratic |x_q - c + t (x_p - x_q)|^2 = r^2 on [0, 1).
    p = W.laplace_sphere()
    g = geometry.from_problem(p)
    c = np.array(p.center)
    r = p.params[0]
    xq = g.coords(g.gamma_minus)
    xp = g.coords(g.gamma_plus[g.partner])
    d = xp - xq
    a = (d * d).sum(1)
    b = 2 * ((xq - c) * d).sum(1)
    cc = ((xq - c) ** 2).sum(1) - r * r
    t_exact = (-b - np.sqrt(b * b - 4 * a * cc)) / (2 * a)
    assert np.abs(g.t - t_exact).max() < 1e-14
    assert np.all((g.t >= 0) & (g.t < 1))
    assert np.abs(np.linalg.norm(g.xstar - c, axis=1) - r).max() < 1e-15
    # the partner is the M+ neighbour with the smallest crossing
    for qi in range(0, len(g.gamma_minus), 7):
        q = g.gamma_minus[qi]
        best = 2.0
        for dd in geometry.DIRS:
            pp = q + dd
            if g.inside[tuple(pp)]:
                xq1, xp1 = g.coords(q), g.coords(pp)
                e = xp1 - xq1
                aa, bb, c2 = e @ e, 2 * (xq1 - c) @ e, (xq1 - c) @ (xq1 - c) - r * r
                best = min(best, (-bb - math.sqrt(bb * bb - 4 * aa * c2)) / (2 * aa))
        assert abs(best - g.t[qi]) < 1e-14


def test_geometry_errors():
    with pytest.raises(geometry.GeometryError):
        geometry.build((9, 9, 9), 1 / 8, (0, 0, 0), "sphere", (0.56, 0.56, 0.56), (0.01,))  # no node inside
    with pytest.raises(geometry.GeometryError):
        geometry.build((9, 9, 9), 1 / 8, (0, 0, 0), "sphere", (0.5, 0.5, 0.5), (0.45,))   # touches the edge
    with pytest.raises(geometry.GeometryError):
        phi = np.full(9 ** 3, np.nan)
        geometry.build((9, 9, 9), 1 / 8, (0, 0, 0), "sampled", phi_nodes=phi)


def test_sampled_level_set_matches_linear_interpolation():
    p = W.laplace_sphere(17)
    X = W.grid_coords(p)
    phi = ((X - 0.5) ** 2).sum(-1) - 0.4 ** 2
    g = geometry.build(p.n, p.h, p.origin, "sampled", phi_nodes=phi)
    ga = geometry.from_problem(p)
    assert np.array_equal(g.gamma_minus, ga.gamma_minus)
    fq = phi[tuple(g.gamma_minus.T)]
    fp = phi[tuple(g.gamma_plus[g.partner].T)]
    assert np.allclose(g.t, fq / (fq - fp), rtol=0, atol=1e-15)
