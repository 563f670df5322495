"""Batched and served solves against the oracle, on problems shaped like the batched workload
(64-96 nodes per axis) whose sums leave the LDS table: sigma = 0 far-field blocks, the
sigma > 0 Yukawa-form far field, global-table gathers (sigma > 0 where that form is not
accepted) and mixed blocks all occur in the batched kernel (asserted from its own pair
classes).  The oracle side is its literal dense operator (one column per gamma- node,
Sec. 3.2) and its own GMRES (Sec. 4), so each problem costs the CPU about a second."""
import math

import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import geometry, gmres, lgf, operators

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def _problem(name, nn, sigma, kind, params, seed):
    rng = np.random.default_rng(seed)
    n, h, o = W.padded_cube(nn)
    c = (0.5, 0.5, 0.5)
    g = W.harmonic_poly(rng.standard_normal(16), c) if sigma == 0.0 else W.yukawa_plane(math.sqrt(sigma),
                                                                                        rng.standard_normal(3))
    return W.Problem(name, n, h, o, float(sigma), kind, c, params, boundary=g)


PROBLEMS = [
    # sigma = 0, offsets to 75: FP32 far blocks beyond the gap, mixed blocks beyond radius 59
    _problem("prolate96", 96, 0.0, "ellipsoid", (0.45, 0.12, 0.12), 9100),
    # sigma = 10 (kappa h = 0.040): the Yukawa-form far field is accepted for FP32
    _problem("yukawa90", 90, 10.0, "ellipsoid", (0.45, 0.1, 0.15), 9101),
    # sigma = 150 (kappa h = 0.148): the form is refused, every far pair is a table gather;
    # offsets to 81 leave whole blocks beyond the LDS radius 59
    _problem("gather100", 100, 150.0, "ellipsoid", (0.47, 0.12, 0.12), 9102),
    _problem("sphere64", 64, 0.0, "sphere", (0.22,), 9103),
    _problem("torus72", 72, 25.0, "torus", (0.25, 0.1), 9104),
]


def oracle_solution(p):
    geo = geometry.from_problem(p)
    assert (geo.d_count() > 0).all()
    G = lgf.LGFTable(geo.max_offset(), p.sigma * p.h ** 2)
    A = operators.dense_operator(geo, G)
    b = p.g(geo.xstar)
    q, _, conv = gmres.gmres(lambda x: A @ x, b, tol=1e-14, maxit=len(b))
    assert conv
    u = operators.double_layer(geo, G, q, operators.gamma_targets(geo))
    return q, u


@pytest.fixture(scope="module")
def oracle():
    return [oracle_solution(p) for p in PROBLEMS]


def contexts():
    out = []
    for p in PROBLEMS:
        c = P.Context.from_problem(p, max_rhs=1, max_krylov=200)
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
        out.append(c)
    return out


def test_the_batch_reaches_every_pair_class():
    ctxs = contexts()
    assert ctxs[1].sizes["far_field_fp32"] == 1 and ctxs[2].sizes["far_field_fp32"] == 0
    with P.Batch(ctxs) as b:
        s32 = b.sum_stats(P.PREC_FP32)
        s64 = b.sum_stats(P.PREC_FP64)
    for c in ctxs:
        c.close()
    assert s32["far_q2"] > 0            # sigma = 0 lattice form and the Yukawa form
    assert s32["far"] > 0               # global-table gathers (the refused Yukawa form)
    assert s32["mixed_far"] > 0 and s32["mixed_near"] > 0
    assert s64["far"] > 0 and s64["mixed_far"] > 0


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_fp64_matches_oracle(oracle, use_graph, tmp_path, monkeypatch):
    monkeypatch.setenv("BAE_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    ctxs = contexts()
    with P.Batch(ctxs) as b:
        res = b.solve(P.SOLVE_FP64, tol=1e-13, use_graph=use_graph)
        assert all(r["converged"] for r in res)
        for p, c, (q0, u0) in zip(PROBLEMS, ctxs, oracle):
            assert rel_l2(c.density(), q0) < 1e-10, p.name
            assert rel_l2(c.gamma_values(), u0) < 1e-10, p.name
    for c in ctxs:
        c.close()


def test_batch_refined_matches_oracle(oracle, tmp_path, monkeypatch):
    monkeypatch.setenv("BAE_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    ctxs = contexts()
    with P.Batch(ctxs) as b:
        b.autotune(P.PREC_FP32)
        res = b.solve(P.SOLVE_FP32_REFINED, tol=1e-11, use_graph=True)
        assert all(r["converged"] for r in res)
        for p, c, (q0, u0) in zip(PROBLEMS, ctxs, oracle):
            assert rel_l2(c.density(), q0) < 1e-8, p.name
            assert rel_l2(c.gamma_values(), u0) < 1e-8, p.name
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("prec,tol,bound", [(P.SOLVE_FP64, 1e-13, 1e-10), (P.SOLVE_FP32_REFINED, 1e-11, 1e-8)])
def test_served_results_match_oracle(oracle, prec, tol, bound):
    with P.Server(hbm_budget=8 << 30, max_slots=3, precision=prec, tol=tol) as srv:
        tickets = [srv.submit_problem(p) for p in PROBLEMS]
        for p, t, (q0, u0) in zip(PROBLEMS, tickets, oracle):
            r, info, q, u = srv.result(t)
            assert r["converged"], (p.name, r)
            assert rel_l2(q, q0) < bound, p.name
            assert rel_l2(u, u0) < bound, p.name
        assert srv.stats()["failed"] == 0
