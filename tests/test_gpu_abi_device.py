"""The C ABI driven from device memory and a caller's stream: right-hand sides from torch
tensors (bae_set_rhs_device), the asynchronous solve ordered on a torch stream
(bae_solve_async / _poll / _wait), device getters, the warm start x0, device-side
non-finite detection, and the server's non-blocking poll.  Results against the oracle."""
import time

import numpy as np
import pytest

import paper_2502_05507_amd as P
import workloads as W
from oracle import bae as obae, box as obox, geometry, sparse

from gpu_common import device, rel_l2, small_problem

pytestmark = pytest.mark.gpu


def test_solve_on_torch_stream_matches_oracle():
    import torch
    dev = device()
    p = W.laplace_sphere()
    ref = obae.solve(p, tol=1e-13)
    s = torch.cuda.Stream()
    with P.Context.from_problem(p) as c:
        xs, _, _ = c.boundary_points()
        g_host = torch.from_numpy(p.g(xs)).pin_memory()
        with torch.cuda.stream(s):
            g = g_host.to(dev, non_blocking=True)
            g = g * 1.0                                   # the caller's own kernel before the solve
            c.set_rhs_device(g, stream=s.cuda_stream)
            c.solve_async(P.SOLVE_FP64, tol=1e-12, stream=s.cuda_stream)
            t0 = time.time()
            while not c.solve_poll():
                assert time.time() - t0 < 60
                time.sleep(0.001)
            res = c.solve_wait(stream=s.cuda_stream)
            q = torch.empty(c.sizes["n_gamma_minus"], dtype=torch.float64, device=dev)
            u = torch.empty(c.sizes["n_targets"], dtype=torch.float64, device=dev)
            c.density_device(q, stream=s.cuda_stream)
            c.gamma_values_device(u, stream=s.cuda_stream)
            u2 = u * 2.0                                  # ordered after the getter on the same stream
        s.synchronize()
        assert res[0]["converged"]
        assert rel_l2(q.cpu().numpy(), ref["q"]) < 1e-10
        assert rel_l2(u.cpu().numpy(), ref["u_gamma"]) < 1e-10
        assert rel_l2(u2.cpu().numpy(), 2 * ref["u_gamma"]) < 1e-10


@pytest.mark.parametrize("particular", ["free", "box"])
def test_device_rhs_with_source_matches_oracle(particular):
    import torch
    dev = device()
    p = W.poisson_ellipsoid(33)
    geo = geometry.from_problem(p)
    u_ref = sparse.solve(geo, 0.0, p.g(geo.xstar), p.f_grid())
    with P.Context.from_problem(p, max_rhs=2) as c:
        xs, _, _ = c.boundary_points()
        G = np.stack([p.g(xs), 2.0 * p.g(xs)])
        F = np.stack([p.f_grid(), 2.0 * p.f_grid()])
        c.set_rhs_device(torch.from_numpy(G).to(dev), torch.from_numpy(F).to(dev), particular=particular)
        res = c.solve(P.SOLVE_FP32_REFINED, tol=1e-12, compute_grid=True)
        assert all(r["converged"] for r in res)
        ug = torch.empty((2, c.sizes["n_targets"]), dtype=torch.float64, device=dev)
        c.gamma_values_device(ug, r=-1)
        ugrid = torch.empty((2,) + tuple(p.n), dtype=torch.float64, device=dev)
        c.solution_device(ugrid, r=-1)
        torch.cuda.synchronize()
        gp, gm, _ = c.sets()
        X = np.concatenate([gp, gm])
        for r in range(2):
            assert rel_l2(ug[r].cpu().numpy(), (r + 1) * u_ref[tuple(X.T)]) < 1e-9
            m = ~np.isnan(u_ref)
            assert rel_l2(ugrid[r].cpu().numpy()[m], (r + 1) * u_ref[m]) < 1e-9
        if particular == "box":
            up = obox.particular_box(geo, 0.0, p.f_grid())
            assert rel_l2(c.particular(0), up) < 1e-12


def test_warm_start():
    import torch
    dev = device()
    p = small_problem("torus", 41, sigma=10.0)
    p.boundary = W.yukawa_plane(np.sqrt(10.0), (1.0, 2.0, 0.5))
    with P.Context.from_problem(p) as c:
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
        r0 = c.solve(P.SOLVE_FP64, tol=1e-12)[0]
        q0 = c.density()
        x0 = torch.from_numpy(q0).to(dev)
        r1 = c.solve(P.SOLVE_FP64, tol=1e-10, x0=x0)[0]     # already converged: no iteration
        assert r1["converged"] and r1["iterations"] == 0
        assert rel_l2(c.density(), q0) < 1e-15
        # continuation: a loose solve's density starts the tight one
        c.solve(P.SOLVE_FP64, tol=1e-5)
        xp = torch.from_numpy(c.density()).to(dev)
        r2 = c.solve(P.SOLVE_FP64, tol=1e-12, x0=xp)[0]
        # (GMRES from a good x0 need not take fewer steps: its residual is the slow part)
        assert r2["converged"] and r2["rel_residual_true"] <= 1e-12 and r2["iterations"] > 0
        assert rel_l2(c.density(), q0) < 1e-10
        r3 = c.solve(P.SOLVE_FP32_REFINED, tol=1e-12, x0=xp)[0]
        assert r3["converged"]
        assert rel_l2(c.density(), q0) < 1e-8


def test_nonfinite_device_input_is_reported():
    import torch
    dev = device()
    p = W.laplace_sphere(17)
    with P.Context.from_problem(p) as c:
        g = torch.ones(c.sizes["n_gamma_minus"], dtype=torch.float64, device=dev)
        g[5] = float("nan")
        c.set_rhs_device(g)
        with pytest.raises(P.BaeError) as e:
            c.solve(P.SOLVE_FP64, tol=1e-10)
        assert e.value.status == -3
        g[5] = 1.0
        c.set_rhs_device(g)
        r = c.solve(P.SOLVE_FP64, tol=1e-12)[0]
        assert r["converged"]
        assert rel_l2(c.density(), np.ones(c.sizes["n_gamma_minus"])) < 1e-10   # g = 1 => q = 1


def test_server_poll():
    p = W.laplace_sphere(25)
    with P.Server(hbm_budget=1 << 32, max_slots=2) as srv:
        t = srv.submit_problem(p)
        states = set()
        t0 = time.time()
        while True:
            st = srv.poll(t)
            states.add(st)
            if st in (2, 3):
                break
            assert time.time() - t0 < 60
            time.sleep(0.001)
        assert st == 2
        r, info, q, u = srv.result(t)
        assert r["converged"]
