"""Serving with continuous batching: every result alone equals the same request solved in
the mix; admission never exceeds the memory budget; oversize requests are refused."""
import threading
import time

import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import geometry

from gpu_common import rel_l2

pytestmark = pytest.mark.gpu


def requests(count=12, seed=8100):
    out = []
    i = 0
    while len(out) < count:
        rng = np.random.default_rng(seed + i)
        nn = int(rng.integers(24, 44))
        p = W.serving_problem(i, nn, seed=seed)
        i += 1
        if (geometry.from_problem(p).d_count() == 0).any():
            continue                       # under-resolved: singular double-layer system
        out.append(p)
    return out


def solo(p, prec):
    with P.Context.from_problem(p, max_rhs=1, max_krylov=200) as c:
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
        r = c.solve(prec, tol=1e-13 if prec == P.SOLVE_FP64 else 1e-11)[0]
        assert r["converged"]
        return c.density(), c.gamma_values(), c.sizes


@pytest.mark.parametrize("prec,threads", [(P.SOLVE_FP64, 1), (P.SOLVE_FP64, 4), (P.SOLVE_FP32_REFINED, 4)])
def test_results_alone_equal_results_in_the_mix(prec, threads):
    probs = requests()
    ref = [solo(p, prec) for p in probs]
    budget = int(sum(z["device_bytes"] for _, _, z in ref) * 0.5)    # forces queueing
    with P.Server(hbm_budget=budget, max_slots=6, precision=prec, setup_threads=threads,
                  tol=1e-13 if prec == P.SOLVE_FP64 else 1e-11) as srv:
        tickets = []
        # staggered arrivals from another thread while earlier requests run
        def feed():
            for p in probs:
                tickets.append(srv.submit_problem(p))
                time.sleep(0.002)
        th = threading.Thread(target=feed)
        th.start()
        th.join()
        admits = []
        for t, (q0, u0, _) in zip(tickets, ref):
            r, info, q, u = srv.result(t)
            assert r["converged"], r
            tol = 1e-10 if prec == P.SOLVE_FP64 else 1e-8
            assert rel_l2(u, u0) < tol and rel_l2(q, q0) < tol
            assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
            admits.append(info["t_admit"])
        # admission is first come, first served, however many set-up threads classify ahead
        assert all(a <= b for a, b in zip(admits, admits[1:])), admits
        st = srv.stats()
        assert st["completed"] == len(probs) and st["failed"] == 0
        assert st["peak_bytes"] <= budget and st["max_active"] <= 6
        assert st["max_active"] >= 2                  # requests really overlapped on the device


def test_oversize_request_is_refused():
    p = requests(1)[0]
    with P.Server(hbm_budget=1 << 20, max_slots=2) as srv:
        t = srv.submit_problem(p)
        with pytest.raises(P.BaeError) as e:
            srv.wait(t)
        assert e.value.status == -7
