"""Seeded, synthetic input generators shared by the tests, the benchmark and the oracle.

This module holds problem *data* only: grid sizes, level-set parameters, seeds, exact
solutions and boundary data.  It contains none of the method's arithmetic (no point
classification, no lattice Green's function, no layer potentials, no Krylov solver);
the oracle and the HIP library each implement those on their own.

Geometry kinds and parameter layout (params vector, length 8):
  sphere     params[0] = radius
  ellipsoid  params[0:3] = semi-axes (a, b, c), axis aligned
  torus      params[0] = R (centre-line radius, in the xy plane), params[1] = r (tube)
  star       params[0] = r0, params[1] = amplitude, params[2] = m, params[3] = k;
             surface radius r0 * (1 + amp * sin(m*theta) * cos(k*phi)),
             theta the polar angle from +z, phi = atan2(y, x)
The interior of every domain is where its level-set function is negative (the
convention of the numerical-results section of the paper).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KINDS = {"sphere": 1, "ellipsoid": 2, "torus": 3, "star": 4, "sampled": 5}


@dataclass
class Problem:
    """One Dirichlet problem -Lap u + sigma u = f in Omega, u = g on the boundary."""
    name: str
    n: tuple            # nodes per axis
    h: float            # grid spacing (isotropic)
    origin: tuple       # coordinates of node (0,0,0)
    sigma: float        # kappa^2 >= 0
    kind: str
    center: tuple
    params: tuple
    exact: object = None        # callable u(x, y, z) or None
    source: object = None       # callable f(x, y, z) or None (f = 0)
    boundary: object = None     # callable g(x, y, z) (defaults to exact)
    nrhs: int = 1
    boundary_rhs: list = field(default_factory=list)  # per-RHS g callables when nrhs > 1
    tol: float = 1e-10

    def params8(self):
        p = list(self.params) + [0.0] * (8 - len(self.params))
        return tuple(float(v) for v in p[:8])

    def g(self, X, r=0):
        """Boundary data of right-hand side r at points X (shape (..., 3))."""
        if self.boundary_rhs:
            fn = self.boundary_rhs[r]
        else:
            fn = self.boundary if self.boundary is not None else self.exact
        return fn(X[..., 0], X[..., 1], X[..., 2])

    def f_grid(self):
        """Source term on the full node grid (n0*n1*n2, k fastest), or None."""
        if self.source is None:
            return None
        X = grid_coords(self)
        return self.source(X[..., 0], X[..., 1], X[..., 2]).reshape(-1)


def grid_coords(p: Problem):
    i = np.arange(p.n[0]) * p.h + p.origin[0]
    j = np.arange(p.n[1]) * p.h + p.origin[1]
    k = np.arange(p.n[2]) * p.h + p.origin[2]
    return np.stack(np.meshgrid(i, j, k, indexing="ij"), axis=-1)


# ----------------------------------------------------------------------------- exact data
def u_c1(x, y, z):
    """Harmonic: exp(x+y) sin(sqrt2 z)."""
    return np.exp(x + y) * np.sin(math.sqrt(2.0) * z)


def u_c2(x, y, z):
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def f_c2(x, y, z):
    return 3.0 * np.pi ** 2 * u_c2(x, y, z)


def yukawa_plane(kappa, a):
    """u = exp(kappa a.x) with |a| = 1 solves -Lap u + kappa^2 u = 0."""
    a = np.asarray(a, dtype=float)
    a = a / np.linalg.norm(a)

    def u(x, y, z):
        return np.exp(kappa * (a[0] * x + a[1] * y + a[2] * z))
    return u


def solid_harmonics(x, y, z):
    """The 16 real solid harmonics of degree <= 3 (unnormalised), stacked on axis 0."""
    return np.stack([
        np.ones_like(x),
        x, y, z,
        x * y, y * z, x * z, x * x - y * y, 2 * z * z - x * x - y * y,
        x * (x * x - 3 * y * y), y * (3 * x * x - y * y), z * (x * x - y * y), x * y * z,
        x * (4 * z * z - x * x - y * y), y * (4 * z * z - x * x - y * y),
        z * (2 * z * z - 3 * x * x - 3 * y * y),
    ])


def harmonic_poly(coeffs, center):
    c = np.asarray(center, dtype=float)

    def g(x, y, z):
        H = solid_harmonics(x - c[0], y - c[1], z - c[2])
        return np.tensordot(np.asarray(coeffs), H, axes=(0, 0))
    return g


# ----------------------------------------------------------------------------- problems
def unit_cube(n_nodes):
    n = int(n_nodes)
    return (n, n, n), 1.0 / (n - 1), (0.0, 0.0, 0.0)


def padded_cube(n_nodes, margin=0.1):
    """Nodes spanning [-margin, 1 + margin]^3, so that radii up to 0.45 about the centre keep
    at least two nodes between the interior and the grid edge even at 32 nodes per axis."""
    n = int(n_nodes)
    return (n, n, n), (1.0 + 2 * margin) / (n - 1), (-margin, -margin, -margin)


def laplace_sphere(n_nodes=33, radius=0.4):
    """Laplace interior Dirichlet on a sphere centred in the unit cube (33^3 at h=1/32)."""
    n, h, o = unit_cube(n_nodes)
    return Problem("laplace_sphere", n, h, o, 0.0, "sphere", (0.5, 0.5, 0.5), (radius,),
                   exact=u_c1, tol=1e-10)


def poisson_ellipsoid(n_nodes=129, axes=(0.45, 0.3, 0.25)):
    """Poisson on an ellipsoid in the unit cube, f from u = sin(pi x) sin(pi y) sin(pi z)."""
    n, h, o = unit_cube(n_nodes)
    return Problem("poisson_ellipsoid", n, h, o, 0.0, "ellipsoid", (0.5, 0.5, 0.5), tuple(axes),
                   exact=u_c2, source=f_c2, tol=1e-10)


def helmholtz_star(n_nodes=257, kappa2=10.0, nrhs=16, seed_base=3000):
    """Modified Helmholtz, kappa^2 = 10, star-shaped domain, nrhs harmonic-polynomial data."""
    n, h, o = unit_cube(n_nodes)
    c = (0.5, 0.5, 0.5)
    rhs = []
    for r in range(nrhs):
        coeffs = np.random.default_rng(seed_base + r).standard_normal(16)
        rhs.append(harmonic_poly(coeffs, c))
    return Problem("helmholtz_star", n, h, o, float(kappa2), "star", c, (0.4, 0.15, 3.0, 2.0),
                   boundary=rhs[0], nrhs=nrhs, boundary_rhs=rhs, tol=1e-10)


def helmholtz_sphere_exact(n_nodes=33, kappa2=10.0, radius=0.4, direction=(1.0, 2.0, 2.0)):
    n, h, o = unit_cube(n_nodes)
    return Problem("helmholtz_sphere", n, h, o, float(kappa2), "sphere", (0.5, 0.5, 0.5), (radius,),
                   exact=yukawa_plane(math.sqrt(kappa2), direction), tol=1e-10)


def batch_problem(i, base_seed=4000):
    """Problem i of the batched workload: seeded sphere/ellipsoid/torus, 32..96 nodes/axis."""
    rng = np.random.default_rng(base_seed + i)
    kind = ["sphere", "ellipsoid", "torus"][int(rng.integers(0, 3))]
    nn = int(rng.integers(32, 97))
    n, h, o = padded_cube(nn)
    c = (0.5, 0.5, 0.5)
    if kind == "sphere":
        params = (float(rng.uniform(0.2, 0.45)),)
    elif kind == "ellipsoid":
        params = tuple(float(v) for v in rng.uniform(0.2, 0.45, 3))
    else:
        rho = float(rng.uniform(0.2, 0.45))
        params = (2.0 * rho / 3.0, rho / 3.0)
    if rng.uniform() < 0.5:
        sigma = 0.0
        g = harmonic_poly(rng.standard_normal(16), c)
    else:
        sigma = float(50.0 - rng.uniform(0.0, 50.0))   # (0, 50]
        a = rng.standard_normal(3)
        g = yukawa_plane(math.sqrt(sigma), a)
    return Problem(f"batch{i}", n, h, o, sigma, kind, c, params, boundary=g, tol=1e-10)


def serving_stream(count, rate, seed=5000):
    """Arrival times (cumulative exponential gaps of mean 1/rate) and problem seeds."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps)
    sizes = np.rint(np.exp(rng.uniform(math.log(32), math.log(256), count))).astype(int)
    return arrivals, sizes


def serving_problem(i, n_nodes, seed=6000):
    rng = np.random.default_rng(seed + i)
    kind = ["sphere", "ellipsoid", "torus", "star"][int(rng.integers(0, 4))]
    n, h, o = padded_cube(n_nodes)
    c = (0.5, 0.5, 0.5)
    if kind == "sphere":
        params = (float(rng.uniform(0.2, 0.45)),)
    elif kind == "ellipsoid":
        params = tuple(float(v) for v in rng.uniform(0.2, 0.45, 3))
    elif kind == "torus":
        rho = float(rng.uniform(0.2, 0.45))
        params = (2.0 * rho / 3.0, rho / 3.0)
    else:
        params = (float(rng.uniform(0.25, 0.38)), 0.15, 3.0, 2.0)
    if rng.uniform() < 0.5:
        sigma = 0.0
        g = harmonic_poly(rng.standard_normal(16), c)
    else:
        sigma = float(50.0 - rng.uniform(0.0, 50.0))
        g = yukawa_plane(math.sqrt(sigma), rng.standard_normal(3))
    return Problem(f"serve{i}", n, h, o, sigma, kind, c, params, boundary=g, tol=1e-10)
