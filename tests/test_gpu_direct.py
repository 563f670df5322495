"""The direct formulation (Sec. 3.1) on the device against the oracle: its operator (the
gamma x gamma LGF sum of Green's third identity plus the Dirichlet rows) and its solves, whose
v on gamma is u_gamma - u_p; u_gamma and the grid solution also against the sparse solve."""
import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import direct, geometry, lgf, operators, sparse

from gpu_common import device, rel_l2, small_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,n,sigma", [("sphere", 33, 0.0), ("torus", 41, 10.0), ("star", 45, 0.0)])
@pytest.mark.parametrize("prec,tol", [(P.PREC_FP64, 1e-10), (P.PREC_FP32, 2e-5)])
def test_direct_operator_matches_oracle(kind, n, sigma, prec, tol):
    import torch
    dev = device()
    p = small_problem(kind, n, sigma)
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), p.sigma * p.h ** 2)
    rng = np.random.default_rng(21)
    v = rng.standard_normal((2, len(g.gamma_plus) + len(g.gamma_minus)))
    with P.Context.from_problem(p, max_rhs=2) as c:
        vt = torch.from_numpy(v).to(dev)
        y = torch.empty_like(vt)
        c.apply_direct(vt, y, prec)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
    for r in range(2):
        ref = direct.direct_apply(g, G, v[r])
        assert rel_l2(y[r], ref) < tol


@pytest.mark.parametrize("make", [lambda: W.laplace_sphere(33), lambda: W.poisson_ellipsoid(33)])
@pytest.mark.parametrize("prec,bound", [(P.SOLVE_FP64, 1e-10), (P.SOLVE_FP32_REFINED, 1e-8)])
def test_direct_solve_matches_oracle(make, prec, bound):
    p = make()
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), 0.0)
    ref = direct.solve(p, g, G, tol=1e-13, grid=True)
    u_sp = sparse.solve(g, 0.0, p.g(g.xstar), p.f_grid())
    with P.Context.from_problem(p) as c:
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs), p.f_grid())
        r = c.solve(prec, tol=1e-12, formulation=P.LAYER_DIRECT, compute_grid=True)[0]
        assert r["converged"], r
        assert rel_l2(c.density(), ref["v"]) < bound
        ug = c.gamma_values()
        assert rel_l2(ug, ref["u_gamma"]) < bound
        T = operators.gamma_targets(g)
        assert rel_l2(ug, u_sp[tuple(T.T)]) < bound
        u = c.solution()
        m = ~np.isnan(u_sp)
        assert np.array_equal(m, ~np.isnan(u))
        assert rel_l2(u[m], u_sp[m]) < bound
        # the double layer reaches the same discrete solution afterwards on the same context
        r2 = c.solve(prec, tol=1e-12)[0]
        assert r2["converged"]
        assert rel_l2(c.gamma_values(), ug) < 10 * bound
