"""GPU parity at the full workload sizes, on outputs the oracle can compute one by one."""
import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import geometry, lgf, operators

from gpu_common import device, rel_l2

pytestmark = pytest.mark.gpu


def test_poisson_ellipsoid_129_matvec_sampled():
    import torch
    p = W.poisson_ellipsoid(129)
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), 0.0)
    T = operators.gamma_targets(g)
    rng = np.random.default_rng(129)
    q = rng.standard_normal(len(g.gamma_minus))
    pick = np.sort(rng.choice(len(T), 300, replace=False))
    ref = operators.double_layer(g, G, q, T[pick])
    with P.Context.from_problem(p) as ctx:
        qd = torch.from_numpy(q).to(device())
        v = torch.empty(len(T), dtype=torch.float64, device=device())
        # FP32: 38% of the pairs take the q = 2 far field, whose dropped term is below 6.1e-7;
        # FFT: the convolution on the 240 x 162 x 135 grid, FP64
        for prec, tol in ((P.PREC_FP64, 1e-10), (P.PREC_FP32, 3e-6), (P.PREC_FFT, 1e-10)):
            ctx.apply_double_layer(qd, v, prec)
            torch.cuda.synchronize()
            err = rel_l2(v.cpu().numpy()[pick], ref)
            print(f"prec {prec}: rel L2 {err:.3e}")
            assert err < tol


def test_poisson_ellipsoid_129_solve_satisfies_oracle_system():
    # The GPU density must solve the oracle's own system b = A q on sampled rows, and its
    # u_gamma must be the oracle's D q + u_p there.
    p = W.poisson_ellipsoid(129)
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), 0.0)
    f = p.f_grid()
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs), f)
        for prec in (P.SOLVE_FP64, P.SOLVE_FP32_REFINED):
            res = ctx.solve(prec, tol=1e-11)[0]
            assert res["converged"]
            q = ctx.density()
            ug = ctx.gamma_values()
            rng = np.random.default_rng(5)
            rows = np.sort(rng.choice(len(g.gamma_minus), 120, replace=False))
            npl = len(g.gamma_plus)
            tq = g.gamma_minus[rows]
            tp = g.gamma_plus[g.partner[rows]]
            pts = np.concatenate([tq, tp])
            v = operators.double_layer(g, G, q, pts)
            up = operators.volume_potential(g, G, f, pts)
            k = len(rows)
            t = g.t[rows]
            Aq = (1 - t) * v[:k] + t * v[k:]
            b = p.g(g.xstar[rows]) - ((1 - t) * up[:k] + t * up[k:])
            bscale = np.abs(p.g(g.xstar)).max()
            assert np.abs(b - Aq).max() < 1e-9 * bscale
            assert np.abs(ug[npl + rows] - (v[:k] + up[:k])).max() < 1e-9 * bscale
            X = g.coords(g.gamma_minus[rows])
            # and the discrete solution is O(h^2) close to the exact one there
            assert np.abs(ug[npl + rows] - p.exact(*X.T)).max() < 2e-3


def test_helmholtz_star_257_sixteen_rhs_sampled():
    import torch
    p = W.helmholtz_star()
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), p.sigma * p.h ** 2)
    T = operators.gamma_targets(g)
    rng = np.random.default_rng(257)
    q = rng.standard_normal((16, len(g.gamma_minus)))
    pick = np.sort(rng.choice(len(T), 24, replace=False))
    ref = np.stack([operators.double_layer(g, G, q[r], T[pick]) for r in range(16)])
    with P.Context.from_problem(p) as ctx:
        z = ctx.sizes
        assert (z["n_gamma_plus"], z["n_gamma_minus"], z["n_ext"], z["n_edges"]) == (114202, 115646, 117098, 212182)
        qd = torch.from_numpy(q).to(device())
        v = torch.empty((16, len(T)), dtype=torch.float64, device=device())
        # FFT: one convolution per right-hand side on the 375 x 480 x 450 grid, FP64
        for prec, tol in ((P.PREC_FP64, 1e-10), (P.PREC_FP32, 2e-5), (P.PREC_FFT, 1e-10)):
            ctx.apply_double_layer(qd, v, prec)
            torch.cuda.synchronize()
            out = v.cpu().numpy()[:, pick]
            for r in range(16):
                assert rel_l2(out[r], ref[r]) < tol
        # kappa^2 h^2 = 1.5e-4: the FP32 sum takes the Yukawa-form far field beyond the LDS
        # radius (all but the nearest pairs); FP64 reads the exact table
        assert ctx.sum_stats(P.PREC_FP32)["far_q2"] > 0.75 * z["n_targets"] * z["n_sources"]
        assert ctx.sum_stats(P.PREC_FP64)["far_q2"] == 0


def test_helmholtz_star_257_refined_solve_satisfies_oracle_system():
    # 16 RHS at once through the matrix-core form, FP32 sum with the Yukawa-form far field
    # plus FP64 refinement: each density must solve the oracle's system b_r = A q_r (exact
    # table) on sampled rows, and converge to the stated tolerance.
    p = W.helmholtz_star()
    g = geometry.from_problem(p)
    s = p.sigma * p.h ** 2
    G = lgf.LGFTable(g.max_offset(), s)
    with P.Context.from_problem(p, max_rhs=16, max_krylov=200) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(np.stack([p.g(xs, r) for r in range(16)]))
        res = ctx.solve(P.SOLVE_FP32_REFINED, tol=1e-10)
        assert all(r["converged"] and r["rel_residual_true"] <= 1e-10 for r in res)
        rng = np.random.default_rng(6)
        rows = np.sort(rng.choice(len(g.gamma_minus), 20, replace=False))
        tq = g.gamma_minus[rows]
        tp = g.gamma_plus[g.partner[rows]]
        pts = np.concatenate([tq, tp])
        t = g.t[rows]
        k = len(rows)
        for r in (0, 7, 15):
            q = ctx.density(r)
            v = operators.double_layer(g, G, q, pts)
            Aq = (1 - t) * v[:k] + t * v[k:]
            b = p.g(g.xstar[rows], r)
            bscale = np.abs(p.g(g.xstar, r)).max()
            assert np.abs(b - Aq).max() < 1e-8 * bscale, (r, np.abs(b - Aq).max() / bscale)
