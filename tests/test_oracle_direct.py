"""Pins of the oracle's direct formulation (Sec. 3.1) to what the paper and the mathematics fix:
the lattice Green's third identity on the plain discrete solution, the equivalence of the
three boundary maps (eq. "equal"), the sparse direct solve, and linear data reproduced exactly."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, geometry, lgf, operators, sparse


def small(kind="sphere", n=13, sigma=0.0, params=None):
    h = 1.0 / (n - 1)
    params = params or {"sphere": (0.3,), "ellipsoid": (0.4, 0.3, 0.25), "torus": (0.26, 0.12),
                        "star": (0.32, 0.15, 3.0, 2.0)}[kind]
    g = geometry.build((n, n, n), h, (0, 0, 0), kind, (0.5, 0.5, 0.5), params)
    G = lgf.LGFTable(g.max_offset() + 1, sigma * h * h)
    return g, G, sigma * h * h


def test_boundary_edges_are_the_cut_edges():
    # every edge joins gamma+ to gamma- at distance 1, and every such pair is listed once
    g, G, s = small("torus", 25)
    e = direct.boundary_edges(g)
    d = np.abs(g.gamma_plus[e[:, 0]] - g.gamma_minus[e[:, 1]]).sum(axis=1)
    assert np.all(d == 1)
    assert len(np.unique(e, axis=0)) == len(e)
    # count independently: cut edges of the M+ indicator along each axis
    ins = g.inside.astype(np.int64)
    cuts = sum(np.abs(np.diff(ins, axis=a)).sum() for a in range(3))
    assert len(e) == cuts


@pytest.mark.parametrize("kind,n,sigma", [("sphere", 15, 0.0), ("torus", 21, 10.0), ("star", 19, 0.0)])
def test_greens_third_identity_on_the_discrete_solution(kind, n, sigma):
    # u from the plain sparse problem (L u = 0 on M+, Dirichlet rows on gamma-): the lattice
    # Green's third identity reproduces u at every node of M+ from its boundary values.
    g, G, s = small(kind, n, sigma)
    rng = np.random.default_rng(11)
    gx = rng.standard_normal(len(g.gamma_minus))
    u = sparse.solve(g, s, gx)
    T = operators.gamma_targets(g)
    v = u[tuple(T.T)]
    rep = direct.representation(g, G, v, g.mplus)
    ref = u[tuple(g.mplus.T)]
    assert np.abs(rep - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kind,n,sigma", [("sphere", 13, 0.0), ("ellipsoid", 15, 30.0)])
def test_three_boundary_maps_agree(kind, n, sigma):
    # eq. "equal": (I - P+)^-1 P- = S+ S-^-1 = D+ D-^-1 (the discrete Dirichlet-to-gamma+ map)
    g, G, s = small(kind, n, sigma)
    assert (g.d_count() > 0).all()
    Pp, Pm = direct.dense_p(g, G)
    M_direct = np.linalg.solve(np.eye(len(Pp)) - Pp, Pm)
    Dp = operators.dense_double_layer(g, G, g.gamma_plus)
    Dm = operators.dense_double_layer(g, G, g.gamma_minus)
    Sp = operators.dense_single_layer(g, G, g.gamma_plus)
    Sm = operators.dense_single_layer(g, G, g.gamma_minus)
    M_double = np.linalg.solve(Dm.T, Dp.T).T
    M_single = np.linalg.solve(Sm.T, Sp.T).T
    scale = np.abs(M_double).max()
    assert np.abs(M_direct - M_double).max() < 1e-11 * scale
    assert np.abs(M_direct - M_single).max() < 1e-11 * scale


@pytest.mark.parametrize("make", [lambda: W.laplace_sphere(17), lambda: W.poisson_ellipsoid(25)])
def test_direct_solve_equals_the_sparse_solve(make):
    p = make()
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), 0.0)
    out = direct.solve(p, g, G, tol=1e-13, grid=True)
    assert out["converged"]
    u = sparse.solve(g, 0.0, p.g(g.xstar), p.f_grid())
    T = operators.gamma_targets(g)
    ref = u[tuple(T.T)]
    assert np.abs(out["u_gamma"] - ref).max() <= 1e-10 * np.abs(ref).max()
    m = ~np.isnan(u)
    assert np.array_equal(m, ~np.isnan(out["u_grid"]))
    assert np.abs(out["u_grid"][m] - u[m]).max() <= 1e-10 * np.abs(u[m]).max()


def test_linear_data_is_reproduced_exactly():
    # sigma = 0: a linear function is lattice-harmonic, so the direct solve returns it on gamma
    g, G, s = small("torus", 21)
    a = np.array([0.3, -1.2, 0.7])
    lin = lambda X: 0.5 + X @ a
    p = W.Problem("lin", g.n, g.h, tuple(g.origin), 0.0, "torus", (0.5, 0.5, 0.5), (0.26, 0.12),
                  boundary=lambda x, y, z: 0.5 + a[0] * x + a[1] * y + a[2] * z)
    out = direct.solve(p, g, G, tol=1e-14)
    T = operators.gamma_targets(g)
    assert np.abs(out["u_gamma"] - lin(g.coords(T))).max() < 1e-11
