"""GPU parity: every step of the HIP path against the FP64 CPU oracle, through the C ABI."""
import math

import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import geometry, gmres, lgf, operators, sparse

from gpu_common import device, oracle_setup, rel_l2, small_problem

pytestmark = pytest.mark.gpu


def torch_mod():
    import torch
    return torch


# ------------------------------------------------------------------ A3: LGF table
@pytest.mark.parametrize("s,R", [(0.0, 40), (0.0, 117), (1.526e-4, 64), (0.0488, 60), (2.0, 24)])
def test_lgf_table_matches_oracle(s, R):
    torch = torch_mod()
    out = torch.empty(P.lgf_table_size(R), dtype=torch.float64, device=device())
    P.lgf_table(s, R, out)
    torch.cuda.synchronize()
    gpu = out.cpu().numpy()
    ref = lgf.LGFTable(R, s).values
    err = np.abs(gpu - ref)
    assert np.all(err <= 1e-13 * np.abs(ref) + 1e-17 * ref[0]), err.max()
    # stencil identity on the device table itself
    t = lgf.LGFTable(R, s, values=gpu)
    n, res = t.stencil_residual()
    assert np.abs(res).max() < 1e-14


def test_lgf_table_watson_value():
    torch = torch_mod()
    out = torch.empty(P.lgf_table_size(2), dtype=torch.float64, device=device())
    P.lgf_table(0.0, 2, out)
    assert abs(out[0].item() - 0.252731009858663003026) < 1e-15


# ------------------------------------------------------------------ A1, A2: point sets and closure
@pytest.mark.parametrize("kind,n", [("sphere", 33), ("ellipsoid", 49), ("torus", 41), ("star", 45)])
def test_sets_and_closure_match_oracle(kind, n):
    p = small_problem(kind, n)
    g = geometry.from_problem(p)
    with P.Context.from_problem(p) as ctx:
        gp, gm, ex = ctx.sets()
        xs, pa, t = ctx.boundary_points()
        z = ctx.sizes
    assert np.array_equal(gp, g.gamma_plus) and np.array_equal(gm, g.gamma_minus) and np.array_equal(ex, g.ext)
    assert np.array_equal(pa, g.partner)
    assert np.abs(t - g.t).max() < 1e-14
    assert np.abs(xs - g.xstar).max() < 1e-14
    assert z["n_mplus"] == g.inside.sum() and z["n_edges"] == len(g.edges)
    assert z["max_offset"] == g.max_offset() and z["n_empty_d"] == int((g.d_count() == 0).sum())


def test_laplace_sphere_sizes():
    with P.Context.from_problem(W.laplace_sphere()) as ctx:
        z = ctx.sizes
    assert (z["n_mplus"], z["n_gamma_plus"], z["n_gamma_minus"], z["n_ext"], z["n_edges"]) == \
        (8733, 1626, 1806, 1994, 3510)


# ------------------------------------------------------------------ A4: kernel values (table / far field)
@pytest.mark.parametrize("prec,tol", [(P.PREC_FP64, 1e-10), (P.PREC_FP32, 2e-6)])
def test_kernel_values_match_oracle(prec, tol):
    torch = torch_mod()
    rng = np.random.default_rng(11)
    off = rng.integers(-117, 118, size=(4000, 3)).astype(np.int32)
    off[:200] = rng.integers(-40, 41, size=(200, 3))
    off[200:206] = [[33, 0, 0], [0, -33, 0], [0, 0, 33], [33, 33, 33], [117, 0, 0], [0, 0, 0]]
    ref = lgf.LGFTable(117, 0.0)(off.astype(np.int64))
    with P.Context.from_problem(W.laplace_sphere()) as ctx:
        o = torch.from_numpy(off).to(device())
        out = torch.empty(len(off), dtype=torch.float64, device=device())
        ctx.lgf_eval(o, out, prec)
        torch.cuda.synchronize()
        gpu = out.cpu().numpy()
    assert np.all(np.abs(gpu - ref) <= tol * ref), np.max(np.abs(gpu - ref) / ref)


@pytest.mark.parametrize("sigma,far32", [(10.0, True), (30.0, True), (200.0, False)])
def test_kernel_values_sigma_positive(sigma, far32):
    """sigma > 0: FP64 reads the exact table everywhere; FP32 uses the Yukawa-form far field
    beyond the LDS radius when the context's check accepts it (small kappa), else the table."""
    torch = torch_mod()
    p = small_problem("sphere", 97, sigma)
    s = sigma * p.h ** 2
    with P.Context.from_problem(p) as ctx:
        R = ctx.sizes["max_offset"]
        rng = np.random.default_rng(12)
        off = rng.integers(-R, R + 1, size=(4000, 3)).astype(np.int32)
        off[:6] = [[R, 0, 0], [0, R, 0], [56, 0, 0], [56, 56, 56], [R, R, R], [0, 0, 0]]
        ref = lgf.LGFTable(R, s)(off.astype(np.int64))
        o = torch.from_numpy(off).to(device())
        out = torch.empty(len(off), dtype=torch.float64, device=device())
        for prec, tol in ((P.PREC_FP64, 1e-13), (P.PREC_FP32, 2e-6 if far32 else 1e-7)):
            ctx.lgf_eval(o, out, prec)
            torch.cuda.synchronize()
            gpu = out.cpu().numpy()
            assert np.all(np.abs(gpu - ref) <= tol * ref), (prec, np.max(np.abs(gpu - ref) / ref))
        st32, st64 = ctx.sum_stats(P.PREC_FP32), ctx.sum_stats(P.PREC_FP64)
    assert st64["far_q2"] == 0
    assert (st32["far_q2"] > 0) == far32


# ------------------------------------------------------------------ A5-A7: double layer and operator
CASES = [("sphere", 33, 0.0), ("ellipsoid", 65, 0.0), ("torus", 41, 10.0), ("sphere", 97, 30.0),
         ("star", 57, 0.0)]


@pytest.mark.parametrize("kind,n,sigma", CASES)
def test_double_layer_matches_oracle(kind, n, sigma):
    torch = torch_mod()
    p = small_problem(kind, n, sigma)
    g, G = oracle_setup(p)
    rng = np.random.default_rng(n)
    q = rng.standard_normal((2, len(g.gamma_minus)))
    T = operators.gamma_targets(g)
    ref = np.stack([operators.double_layer(g, G, q[r], T) for r in range(2)])
    with P.Context.from_problem(p) as ctx:
        qd = torch.from_numpy(q).to(device())
        v = torch.empty((2, len(T)), dtype=torch.float64, device=device())
        ctx.apply_double_layer(qd, v, P.PREC_FP64)
        torch.cuda.synchronize()
        v64 = v.cpu().numpy()
        ctx.apply_double_layer(qd, v, P.PREC_FP32)
        torch.cuda.synchronize()
        v32 = v.cpu().numpy()
    for r in range(2):
        assert rel_l2(v64[r], ref[r]) < 1e-10
        assert rel_l2(v32[r], ref[r]) < 2e-5


@pytest.mark.parametrize("kind,n,sigma", CASES[:3])
def test_operator_matches_oracle(kind, n, sigma):
    torch = torch_mod()
    p = small_problem(kind, n, sigma)
    g, G = oracle_setup(p)
    rng = np.random.default_rng(3 * n)
    q = rng.standard_normal(len(g.gamma_minus))
    ref = operators.bae_apply(g, G, q)
    with P.Context.from_problem(p) as ctx:
        qd = torch.from_numpy(q).to(device())
        aq = torch.empty_like(qd)
        ctx.apply_operator(qd, aq, P.PREC_FP64)
        torch.cuda.synchronize()
        assert rel_l2(aq.cpu().numpy(), ref) < 1e-10


def test_gauss_law_on_device():
    # (D 1)(m) = 1 on gamma for sigma = 0: a pin that needs no oracle arithmetic
    torch = torch_mod()
    p = W.poisson_ellipsoid(129)
    with P.Context.from_problem(p) as ctx:
        m = ctx.sizes["n_gamma_minus"]
        one = torch.ones(m, dtype=torch.float64, device=device())
        v = torch.empty(ctx.sizes["n_targets"], dtype=torch.float64, device=device())
        ctx.apply_double_layer(one, v, P.PREC_FP64)
        torch.cuda.synchronize()
        assert (v - 1).abs().max().item() < 1e-9


# ------------------------------------------------------------------ A8: solves
def oracle_solution(p, g, G, tol=1e-13):
    gx = p.g(g.xstar)
    f = p.f_grid()
    b = operators.rhs(g, G, gx, f)
    q, hist, conv = gmres.gmres(lambda x: operators.bae_apply(g, G, x), b, tol=tol)
    T = operators.gamma_targets(g)
    ug = operators.double_layer(g, G, q, T)
    if f is not None:
        ug = ug + operators.volume_potential(g, G, f, T)
    return q, ug, hist


@pytest.mark.parametrize("prec,tol_q", [(P.SOLVE_FP64, 1e-10), (P.SOLVE_FP32_REFINED, 1e-8)])
def test_laplace_sphere_solve_matches_oracle(prec, tol_q):
    p = W.laplace_sphere()
    g, G = oracle_setup(p)
    q_ref, ug_ref, hist_ref = oracle_solution(p, g, G)
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs))
        res = ctx.solve(prec, tol=1e-13)
        q = ctx.density()
        ug = ctx.gamma_values()
        hist = ctx.history()
    assert res[0]["converged"] and res[0]["rel_residual_true"] < 1e-12
    assert rel_l2(q, q_ref) < tol_q and rel_l2(ug, ug_ref) < tol_q
    if prec == P.SOLVE_FP64:
        # Givens residual estimates agree over the first iterations (rounding differs later)
        k = min(10, len(hist), len(hist_ref))
        assert np.allclose(hist[:k], hist_ref[:k], rtol=1e-6)


def test_poisson_with_source_and_grid_output():
    p = W.poisson_ellipsoid(33)
    g, G = oracle_setup(p)
    q_ref, ug_ref, _ = oracle_solution(p, g, G)
    us = sparse.solve(g, 0.0, p.g(g.xstar), p.f_grid())
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs), p.f_grid())
        res = ctx.solve(P.SOLVE_FP64, tol=1e-13, compute_grid=True)
        ug = ctx.gamma_values()
        u = ctx.solution()
    assert res[0]["converged"]
    assert rel_l2(ug, ug_ref) < 1e-10
    nplus = ~np.isnan(us)
    assert np.array_equal(~np.isnan(u), nplus)
    assert np.abs(u[nplus] - us[nplus]).max() < 1e-10 * np.abs(us[nplus]).max()


def test_helmholtz_multi_rhs_and_refinement():
    p = small_problem("torus", 41, 10.0)
    g, G = oracle_setup(p)
    rng = np.random.default_rng(99)
    coeffs = rng.standard_normal((3, 16))
    gs = [W.harmonic_poly(c, (0.5, 0.5, 0.5)) for c in coeffs]
    refs = []
    for fn in gs:
        b = fn(*g.xstar.T)
        q, _, _ = gmres.gmres(lambda x: operators.bae_apply(g, G, x), b, tol=1e-13)
        refs.append(q)
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        G3 = np.stack([fn(*xs.T) for fn in gs])
        ctx.set_rhs(G3)
        for prec, tol_q in ((P.SOLVE_FP64, 1e-10), (P.SOLVE_FP32_REFINED, 1e-8)):
            res = ctx.solve(prec, tol=1e-12)
            assert all(r["converged"] for r in res)
            for r in range(3):
                assert rel_l2(ctx.density(r), refs[r]) < tol_q


# ------------------------------------------------------------------ failure handling
def test_error_paths():
    p = W.laplace_sphere(17)
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        with pytest.raises(P.BaeError):
            ctx.solve()                                   # before set_rhs
        bad = p.g(xs)
        bad[3] = np.nan
        with pytest.raises(P.BaeError) as e:
            ctx.set_rhs(bad)
        assert e.value.status == -3
        ctx.set_rhs(p.g(xs))
        res = ctx.solve(P.SOLVE_FP64, tol=1e-14, maxit=2)
        assert res[0]["status"] == 1 and not res[0]["converged"] and res[0]["iterations"] == 2
    with pytest.raises(P.BaeError) as e:
        P.Context((17, 17, 17), 1 / 16, (0, 0, 0), 0.0, "sphere", (0.5, 0.5, 0.5), (0.49,))
    assert e.value.status == -2


def test_sum_alone_for_timing_leaves_the_operator_unchanged():
    """bae_lgf_sum_repeat (the sum kernel alone, for timing) rejects bad counts and leaves
    the operator's results exactly as they were."""
    torch = torch_mod()
    p = W.laplace_sphere(33)
    with P.Context.from_problem(p) as ctx:
        z = ctx.sizes
        q = torch.from_numpy(np.random.default_rng(3).standard_normal(z["n_gamma_minus"])).to(device())
        v0 = torch.empty(z["n_targets"], dtype=torch.float64, device=device())
        v1 = torch.empty_like(v0)
        for prec in (P.PREC_FP64, P.PREC_FP32):
            ctx.apply_double_layer(q, v0, prec)
            ctx.lgf_sum_repeat(q, 5, prec)
            ctx.apply_double_layer(q, v1, prec)
            torch.cuda.synchronize()
            assert torch.equal(v0, v1)
        for bad in (0, 1001):
            with pytest.raises(P.BaeError) as e:
                ctx.lgf_sum_repeat(q, bad)
            assert e.value.status == -1


# ------------------------------------------------------------------ Algorithm 1: box particular solution
@pytest.mark.parametrize("kind,n,sigma", [("ellipsoid", 33, 0.0), ("torus", 41, 10.0)])
def test_box_particular_solution_matches_oracle(kind, n, sigma):
    """u_p = G_h[chi_{M+} f] on the finite grid (sine transforms on the device) against the
    oracle's; the solve on it gives the free-space path's u_gamma and grid solution."""
    from oracle import box
    p = small_problem(kind, n, sigma)
    g = geometry.from_problem(p)
    X = g.coords(np.indices(g.n).reshape(3, -1).T)
    f = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] + 1.0).reshape(-1)
    ref = box.particular_box(g, sigma * p.h ** 2, f)
    gx_fn = lambda Y: np.cos(Y[:, 0]) * Y[:, 1] + Y[:, 2]
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(gx_fn(xs), f, particular="box")
        up = ctx.particular()
        assert np.abs(up - ref).max() < 1e-12 * np.abs(ref).max(), np.abs(up - ref).max() / np.abs(ref).max()
        rb = ctx.solve(P.SOLVE_FP64, tol=1e-13, compute_grid=True)[0]
        ug_b, u_b = ctx.gamma_values(), ctx.solution()
        ctx.set_rhs(gx_fn(xs), f)
        rf = ctx.solve(P.SOLVE_FP64, tol=1e-13, compute_grid=True)[0]
        ug_f, u_f = ctx.gamma_values(), ctx.solution()
    assert rb["converged"] and rf["converged"]
    assert rel_l2(ug_b, ug_f) < 1e-10
    nplus = ~np.isnan(u_f)
    assert np.array_equal(~np.isnan(u_b), nplus)
    assert np.abs(u_b[nplus] - u_f[nplus]).max() < 1e-10 * np.abs(u_f[nplus]).max()


# ------------------------------------------------------------------ single-layer formulation
@pytest.mark.parametrize("kind,n,sigma", [("sphere", 33, 0.0), ("torus", 41, 10.0)])
def test_single_layer_matches_oracle(kind, n, sigma):
    """Sec. 3.4: v = [S+ q; S- q], S(m,n) = G(m - n) on gamma- sources, against the oracle."""
    torch = torch_mod()
    p = small_problem(kind, n, sigma)
    g, G = oracle_setup(p)
    q = np.random.default_rng(5 * n).standard_normal((2, len(g.gamma_minus)))
    T = operators.gamma_targets(g)
    ref = q @ operators.dense_single_layer(g, G, T).T
    with P.Context.from_problem(p, max_rhs=2) as ctx:
        qd = torch.from_numpy(q).to(device())
        v = torch.empty((2, len(T)), dtype=torch.float64, device=device())
        for prec, tol in ((P.PREC_FP64, 1e-10), (P.PREC_FP32, 2e-5)):
            ctx.apply_single_layer(qd, v, prec)
            torch.cuda.synchronize()
            out = v.cpu().numpy()
            for r in range(2):
                assert rel_l2(out[r], ref[r]) < tol, (prec, r, rel_l2(out[r], ref[r]))


def test_single_layer_solve_reaches_the_double_layer_solution():
    """Sec. 3.4: (Phi+ S+ + Phi- S-) q_s = b.  Its density against the oracle's GMRES on the
    same system; u_gamma and u on N+ equal the double-layer solve's (both are the discrete
    solution); afterwards the operator is the double layer again."""
    torch = torch_mod()
    p = W.poisson_ellipsoid(33)
    g, G = oracle_setup(p)
    T = operators.gamma_targets(g)
    b = operators.rhs(g, G, p.g(g.xstar), p.f_grid())
    qs_ref, _, conv = gmres.gmres(lambda x: operators.closure(g, operators.single_layer(g, G, x, T)), b, tol=1e-13)
    assert conv
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs), p.f_grid())
        rd = ctx.solve(P.SOLVE_FP64, tol=1e-13, compute_grid=True)[0]
        ug_d, u_d = ctx.gamma_values(), ctx.solution()
        nplus = ~np.isnan(u_d)
        for prec, tol, tq, tu in ((P.SOLVE_FP64, 1e-13, 1e-9, 1e-10), (P.SOLVE_FP32_REFINED, 1e-10, 1e-6, 1e-8)):
            rs = ctx.solve(prec, tol=tol, compute_grid=True, formulation=P.LAYER_SINGLE)[0]
            assert rs["converged"], rs
            qs, ug_s, u_s = ctx.density(), ctx.gamma_values(), ctx.solution()
            print(f"single layer ({prec}): {rs['iterations']} iterations; double layer {rd['iterations']}")
            assert rel_l2(qs, qs_ref) < tq, rel_l2(qs, qs_ref)
            assert rel_l2(ug_s, ug_d) < tu, rel_l2(ug_s, ug_d)
            assert np.array_equal(~np.isnan(u_s), nplus)
            assert np.abs(u_s[nplus] - u_d[nplus]).max() < tu * np.abs(u_d[nplus]).max()
        q = np.random.default_rng(8).standard_normal(len(g.gamma_minus))
        qd = torch.from_numpy(q).to(device())
        aq = torch.empty_like(qd)
        ctx.apply_operator(qd, aq, P.PREC_FP64)
        torch.cuda.synchronize()
        assert rel_l2(aq.cpu().numpy(), operators.bae_apply(g, G, q)) < 1e-10


# ------------------------------------------------------------------ the largest lattice offsets
class _EntryLGF:
    """The oracle's G_0 entry by entry (its tables would need every offset up to 2046)."""

    def __init__(self):
        self.cache = {}

    def pairs(self, m, s):
        d = np.abs(np.asarray(m)[:, None, :] - np.asarray(s)[None, :, :])
        d.sort(axis=2)
        u, inv = np.unique(d.reshape(-1, 3), axis=0, return_inverse=True)
        vals = np.array([self.cache[k] if k in self.cache else self.cache.setdefault(k, lgf.lgf_entry(np.array(k), 0.0))
                         for k in map(tuple, u)])
        return vals[inv.reshape(-1)].reshape(d.shape[:2])


def test_largest_lattice_offsets_two_balls():
    """Two small balls at the two ends of a 2049-node axis (a sampled level set): offsets
    up to 2046, lattice coordinates up to 2048, the limit of the FP32 path's binary16
    differences and of its matrix-core offset forms (16 right-hand sides: the far blocks of
    the blocked kernel).  Double layer against the oracle's entry-by-entry LGF."""
    torch = torch_mod()
    n, h = (2049, 11, 11), 1.0 / 64
    idx = np.indices(n).reshape(3, -1).T.astype(float)
    c1, c2, r = np.array([5.0, 5.0, 5.0]), np.array([2043.0, 5.0, 5.0]), 2.6
    phi = (np.minimum(np.linalg.norm(idx - c1, axis=1), np.linalg.norm(idx - c2, axis=1)) - r) * h
    g = geometry.build(n, h, (0.0, 0.0, 0.0), "sampled", phi_nodes=phi)
    assert g.max_offset() == 2046
    T = operators.gamma_targets(g)
    D = operators.dense_double_layer(g, _EntryLGF(), T)
    nr = 16
    q = np.random.default_rng(21).standard_normal((nr, len(g.gamma_minus)))
    ref = q @ D.T
    with P.Context(n, h, (0.0, 0.0, 0.0), 0.0, "sampled", phi=phi, max_rhs=nr) as ctx:
        z = ctx.sizes
        assert (z["n_gamma_plus"], z["n_gamma_minus"], z["n_ext"], z["max_offset"]) == \
            (len(g.gamma_plus), len(g.gamma_minus), len(g.ext), 2046)
        assert ctx.sum_stats(P.PREC_FP32)["far_q2"] > 0      # the binary16 far field runs
        qd = torch.from_numpy(q).to(device())
        v = torch.empty((nr, len(T)), dtype=torch.float64, device=device())
        # the FFT convolution runs on a box 2043 nodes long: transform length 4096 along x
        for prec, tol in ((P.PREC_FP64, 1e-10), (P.PREC_FP32, 2e-5), (P.PREC_FFT, 1e-10)):
            ctx.apply_double_layer(qd, v, prec)
            torch.cuda.synchronize()
            out = v.cpu().numpy()
            for rr in range(nr):
                assert rel_l2(out[rr], ref[rr]) < tol, (prec, rr, rel_l2(out[rr], ref[rr]))
        assert ctx.get_sizes()["conv_fft"][0] >= 2 * ctx.get_sizes()["conv_box"][0] - 1 > 4000
        # the box particular solution on this long, thin box (a 2047-point sine transform,
        # FFT length 4096); without it there is no u_p to read
        from oracle import box
        ctx.set_rhs(np.zeros(len(g.gamma_minus)), np.ones(int(np.prod(n))), particular="box")
        ref_p = box.particular_box(g, 0.0, np.ones(int(np.prod(n))))
        assert np.abs(ctx.particular() - ref_p).max() < 1e-12 * np.abs(ref_p).max()
        ctx.set_rhs(np.zeros(len(g.gamma_minus)), np.ones(int(np.prod(n))))
        with pytest.raises(P.BaeError):
            ctx.particular()


@pytest.mark.parametrize("n", [(41, 36, 29), (39, 44, 35)])
def test_box_on_non_cubic_grids(n):
    """Sine transforms of lengths whose FFTs take radices 4, 2, 5, 7 and the primes 17, 19, 43:
    u_p against the oracle's (scipy DST-I) and Algorithm 1's reconstruction of u on the grid
    against the sparse solve."""
    from oracle import box, sparse
    h = 1.0 / 40
    c = tuple(0.5 * (v - 1) * h for v in n)
    p = W.Problem("box", n, h, (0.0, 0.0, 0.0), 20.0, "ellipsoid", c, (0.33, 0.36, 0.29))
    g = geometry.from_problem(p)
    X = g.coords(np.indices(g.n).reshape(3, -1).T)
    f = (np.cos(3 * X[:, 0]) + X[:, 1] * X[:, 2] ** 2 + 0.5).reshape(-1)
    gx_fn = lambda Y: np.sin(Y[:, 0] + 2 * Y[:, 1]) + Y[:, 2]
    s = p.sigma * h * h
    ref_p = box.particular_box(g, s, f)
    u_ref = sparse.solve(g, s, gx_fn(g.xstar), f)
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        for particular in ("box", "free"):
            ctx.set_rhs(gx_fn(xs), f, particular=particular)
            if particular == "box":
                up = ctx.particular()
                assert np.abs(up - ref_p).max() < 1e-12 * np.abs(ref_p).max()
            r = ctx.solve(P.SOLVE_FP64, tol=1e-13, compute_grid=True)[0]
            assert r["converged"]
            u = ctx.solution()
            m = ~np.isnan(u_ref)
            assert np.array_equal(~np.isnan(u), m)
            assert np.abs(u[m] - u_ref[m]).max() < 1e-10 * np.abs(u_ref[m]).max(), particular


# ------------------------------------------------------------------ A10: 16 right-hand sides (MFMA form)
@pytest.mark.parametrize("kind,n,sigma", [("ellipsoid", 65, 0.0), ("sphere", 97, 0.0), ("sphere", 97, 30.0),
                                          ("torus", 41, 10.0)])
def test_sixteen_rhs_blocked_form_matches_oracle(kind, n, sigma):
    torch = torch_mod()
    p = small_problem(kind, n, sigma)
    g, G = oracle_setup(p)
    rng = np.random.default_rng(7 * n)
    nr = 23                                   # a 16-wide MFMA group, a 4-RHS VALU launch, 3 single ones
    q = rng.standard_normal((nr, len(g.gamma_minus)))
    T = operators.gamma_targets(g)
    D = operators.dense_double_layer(g, G, T) if len(T) * len(g.gamma_minus) < 3e7 else None
    pick = rng.choice(len(T), size=min(len(T), 400), replace=False)
    ref = q @ (D if D is not None else operators.dense_double_layer(g, G, T[pick])).T
    with P.Context.from_problem(p, max_rhs=nr) as ctx:
        far = ctx.sum_stats(P.PREC_FP32)["far_q2"]
        if sigma == 0.0:
            # all pairs within the LDS table at 65^3; at 97^3 some lie beyond the far-field gap,
            # so the matrix-core kernel's FP32 far-block loop runs
            assert (far > 0) == (n > 65), far
        qd = torch.from_numpy(q).to(device())
        v = torch.empty((nr, len(T)), dtype=torch.float64, device=device())
        for prec, tol in ((P.PREC_FP64, 1e-10), (P.PREC_FP32, 2e-5)):
            ctx.apply_double_layer(qd, v, prec)
            torch.cuda.synchronize()
            out = v.cpu().numpy()
            if D is None:
                out = out[:, pick]
            for r in range(nr):
                assert rel_l2(out[r], ref[r]) < tol, (prec, r, rel_l2(out[r], ref[r]))


# ------------------------------------------------------------------ A9: refinement with Krylov recycling
@pytest.mark.parametrize("kind,n,sigma,nr", [("sphere", 33, 0.0, 1), ("torus", 41, 10.0, 3)])
def test_refined_solve_with_recycling_matches_oracle(kind, n, sigma, nr):
    """The later inner solves of a refined solve, augmented with the first one's Krylov space
    (forced on here; automatic only for long matvecs), reach the oracle's FP64 densities, in
    no more iterations than plain restarts."""
    p = small_problem(kind, n, sigma)
    g, G = oracle_setup(p)
    rng = np.random.default_rng(17 * n)
    gs = [W.harmonic_poly(c, (0.5, 0.5, 0.5)) for c in rng.standard_normal((nr, 16))]
    refs = [gmres.gmres(lambda x: operators.bae_apply(g, G, x), fn(*g.xstar.T), tol=1e-13)[0] for fn in gs]
    with P.Context.from_problem(p, max_rhs=nr) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(np.stack([fn(*xs.T) for fn in gs]))
        plain = ctx.solve(P.SOLVE_FP32_REFINED, tol=1e-10, recycle_dim=-1)
        res = ctx.solve(P.SOLVE_FP32_REFINED, tol=1e-10, recycle_dim=32)
        for r in range(nr):
            assert res[r]["converged"] and res[r]["rel_residual_true"] <= 1e-10
            assert res[r]["iterations"] <= plain[r]["iterations"], (res[r]["iterations"], plain[r]["iterations"])
            assert rel_l2(ctx.density(r), refs[r]) < 1e-8, (r, rel_l2(ctx.density(r), refs[r]))
