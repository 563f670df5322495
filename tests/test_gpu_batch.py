"""Batched lock-step solves (graph-captured and eager) against solo solves of the same problems."""
import os

import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import geometry

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def make_problems(count=10, base_seed=7000):
    """Seeded small problems; geometries whose grid leaves a gamma- node with an empty D_n
    (a singular, possibly inconsistent double-layer system) are redrawn."""
    probs = []
    i = 0
    while len(probs) < count:
        rng = np.random.default_rng(base_seed + i)
        nn = int(rng.integers(24, 41))
        p = W.batch_problem(i, base_seed=base_seed)
        n, h, o = W.padded_cube(nn, margin=0.15)
        p.n, p.h, p.origin = n, h, o
        i += 1
        if (geometry.from_problem(p).d_count() == 0).any():
            continue
        probs.append(p)
    return probs


def contexts(probs):
    out = []
    for p in probs:
        c = P.Context.from_problem(p, max_rhs=1, max_krylov=150)
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
        out.append(c)
    return out


@pytest.fixture(scope="module")
def solo():
    probs = make_problems()
    ctxs = contexts(probs)
    ref = []
    for c in ctxs:
        r = c.solve(P.SOLVE_FP64, tol=1e-12)[0]
        assert r["converged"]
        ref.append((c.density(), c.gamma_values()))
    for c in ctxs:
        c.close()
    return probs, ref


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_fp64_equals_solo(solo, use_graph, tmp_path):
    os.environ["BAE_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")
    probs, ref = solo
    ctxs = contexts(probs)
    with P.Batch(ctxs) as b:
        for replay in range(3):      # graph replays, with eager host work in between
            res = b.solve(P.SOLVE_FP64, tol=1e-12, use_graph=use_graph)
            assert all(r["converged"] for r in res)
            for c, (q, ug) in zip(ctxs, ref):
                assert rel_l2(c.density(), q) < 1e-10
                assert rel_l2(c.gamma_values(), ug) < 1e-10
                c.history()
    for c in ctxs:
        c.close()


def test_batch_refined_and_autotune(solo, tmp_path):
    os.environ["BAE_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")
    probs, ref = solo
    ctxs = contexts(probs)
    with P.Batch(ctxs) as b:
        chosen = b.autotune(P.PREC_FP32)
        # the tuner times every (blocks per chunk, grid multiplier) candidate and keeps the fastest
        assert chosen["blocks_per_chunk"] in (2, 4, 8, 16, 32, 64) and chosen["grid_multiplier"] in (1, 2, 4)
        res = b.solve(P.SOLVE_FP32_REFINED, tol=1e-11, use_graph=True)
        assert all(r["converged"] for r in res)
        for c, (q, ug) in zip(ctxs, ref):
            assert rel_l2(c.gamma_values(), ug) < 1e-8
    assert os.path.exists(tmp_path / "tune.txt")
    # a new batch of the same size class picks the cached tiling up
    with P.Batch(ctxs) as b2:
        res = b2.solve(P.SOLVE_FP64, tol=1e-12)
        assert all(r["converged"] for r in res)
    for c in ctxs:
        c.close()
