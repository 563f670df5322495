#!/usr/bin/env python3
"""Benchmark of the unfitted-BAE hot path on one MI355X.

Default workload (the JSON line the contract asks for): Poisson -Lap u = f on the ellipsoid
with semi-axes (0.45, 0.3, 0.25) centred in the unit cube, h = 1/128 (129^3 nodes), f and g
from u = sin(pi x) sin(pi y) sin(pi z).  One step = one complete solve on device-resident
inputs: FP64 iterative refinement around GMRES with the FP32 LGF sum (every matvec =
double-layer weights, the LGF sum over |gamma| x |gamma- u E| pairs, the closure) and the FP64
residual matvecs, the last of which also gives u_gamma.  value = LGF pair-interactions
evaluated in the timed steps divided by their wall time.  Also reported: solves/s and p50/p99
latency of the refined and of the plain FP64 path, matvec-only rates (HIP events on the launch
stream), the roofline of the FP32 LGF-sum kernel (its operations and flops counted per pair
class, over the kernel's own duration: HIP events around back-to-back launches of the sum
alone), and the CPU oracle's rate on a bounded sample of the same matvec.

Other workloads (--workload; their own JSON line, not the contract's):
  laplace_sphere   33^3 Laplace sphere, FP64 and refined solve latency
  helmholtz_star   257^3 modified Helmholtz, 16 right-hand sides (MFMA form), refined
  batch            512 seeded small problems in one lock-step, graph-replayed batch
  serve            Poisson arrivals into the continuous-batching server, p50/p99 latency
  profile          matvecs only (for rocprofv3) plus a device copy of known size
  formulations     single- against double-layer formulation (iterations, time) at 129^3
  particular       free-space against finite-grid (sine-transform) particular solution at 129^3
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LGF pair-interactions/s per BAE matvec; solves/s + p99 latency at rel err ≤1e-8"
PEAK_FP32_VECTOR = 157.3   # TFLOP/s, MI355X published FP32 vector peak (packed FP32 included)
PEAK_FP64_VECTOR = 78.6    # TFLOP/s
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one lane-operation per lane and
# clock (an FMA is one operation; its two flops make 78.6 TFLOP/s non-packed)
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9 / 1e12
# flops per pair (kernel value + one accumulate) by the kernel's pair classes
FLOPS = {"fp32": {"near": 2, "far": 23, "far_q2": 23, "mixed_near": 2, "mixed_far": 23},
         "fp64": {"near": 2, "far": 46, "far_q2": 46, "mixed_near": 2, "mixed_far": 46}}
# VALU lane-operations per pair the evaluation needs, by pair class:
#   table lookup: 3 |t - s| + min/median/max + index add (+ a shift in FP64) + accumulate
#   far field, FP64 (q = 4): 3 differences, 3 squares, r^2, e2 and e3, the rsqrt estimate
#     and its Newton step, the rho powers and invariants, the polynomial, the product with
#     1/|n| and the accumulate
#   far field, FP32 (q = 2): the packed binary16 (x, y) difference, the z difference and its
#     square, two dot products (|n|^2 and n_y^2 - n_x^2), rsqrt, rho, the two ratios, the
#     four-term polynomial, the product with 1/|n| and the accumulate
#   mixed pairs: the chosen path plus the per-pair test
OPS = {"fp32": {"near": 8, "far": 19, "far_q2": 15, "mixed_near": 10, "mixed_far": 24},
       "fp64": {"near": 9, "far": 37, "far_q2": 37, "mixed_near": 11, "mixed_far": 42}}


# HBM bytes per launch of the FP32 LGF-sum kernel on this workload, from rocprofv3 FETCH_SIZE
# (x2.00) and WRITE_SIZE (x1.00) runs calibrated on 256 MiB copies
# (profiles/lgf_sum_poisson_ellipsoid_129_counters.md); valid only for the kernel sources
# it was measured on, identified by their hash.
MEASURED_TRAFFIC = {"sources_sha256_16": "c8628c25f06815ff", "bytes": (12255.2 * 2.0 + 18518.7 * 1.0) * 1024}
KERNEL_SOURCES = ("paper_2502_05507_amd/csrc/lgf_sum.hip", "paper_2502_05507_amd/csrc/lgf_device.hpp")


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_of(stats, prec, nrhs=1, gathers=False):
    """Algorithmic flops of one launch: far-field pairs count their formula, table lookups
    (near pairs; with sigma > 0 every pair) only the accumulate."""
    per = {k: 2 for k in FLOPS[prec]} if gathers else FLOPS[prec]
    tot = sum(stats[k] * per[k] for k in per)
    return tot + (nrhs - 1) * 2 * sum(stats.values())


def ops_of(stats, prec):
    """VALU lane-operations of one launch (OPS per pair class)."""
    return sum(stats[k] * OPS[prec][k] for k in OPS[prec])


def time_applies(torch, ctx, q, v, prec, reps):
    stream = torch.cuda.current_stream()
    for _ in range(3):
        ctx.apply_double_layer(q, v, prec)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.apply_double_layer(q, v, prec)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    return float(np.median(times))


def time_sum_kernel(torch, ctx, q, prec, reps, burst=20):
    """Average duration of the LGF-sum kernel alone: HIP events on the launch stream around
    1 and 1 + burst back-to-back launches (bae_lgf_sum_repeat, which forms the weights once
    first); the difference over burst removes the weights launch and the event overhead."""
    stream = torch.cuda.current_stream()

    def timed(n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.lgf_sum_repeat(q, n, prec)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    timed(2)
    per = [(timed(1 + burst) - timed(1)) / burst for _ in range(reps)]
    return float(np.median(per))


def cpu_baseline(p, budget_s=12.0):
    """The oracle's literal double-layer sum on a bounded sample of targets (1 thread)."""
    from oracle import geometry, lgf, operators
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), p.sigma * p.h ** 2)
    rng = np.random.default_rng(1234)
    q = rng.standard_normal(len(g.gamma_minus))
    T = operators.gamma_targets(g)
    n_src = len(g.gamma_minus) + len(g.ext)
    order = rng.permutation(len(T))
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < len(T):
        blk = T[order[done:done + 64]]
        operators.double_layer(g, G, q, blk)
        done += len(blk)
    dt = time.perf_counter() - t0
    return {"value": done * n_src / dt, "unit": "pair-interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of {len(T)} gamma targets x {n_src} sources (literal double-layer sum, FP64, "
                      f"NumPy single thread), {dt:.1f} s"}


def headline(args, torch, P, W):
    dev = torch.device("cuda:0")
    p = W.poisson_ellipsoid(args.nodes)
    t_setup = time.perf_counter()
    ctx = P.Context.from_problem(p)
    xs, _, _ = ctx.boundary_points()
    ctx.set_rhs(p.g(xs), p.f_grid())
    t_setup = time.perf_counter() - t_setup
    z = ctx.sizes
    pairs_mv = z["n_targets"] * z["n_sources"]
    log(f"setup {t_setup:.2f}s sizes {z}")

    tol = 1e-10
    for _ in range(args.warmup):
        ctx.solve(P.SOLVE_FP32_REFINED, tol=tol)
    torch.cuda.synchronize()
    lat, pairs_total = [], 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        r = ctx.solve(P.SOLVE_FP32_REFINED, tol=tol)[0]
        lat.append(time.perf_counter() - s0)
        pairs_total += (r["matvecs_fp64"] + r["matvecs_fp32"]) * pairs_mv
        log(f"step {k}: {lat[-1] * 1e3:.1f} ms, iters {r['iterations']}, outer {r['outer_steps']}, "
            f"relres {r['rel_residual_true']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    refined = r
    u32 = ctx.gamma_values()

    ctx.solve(P.SOLVE_FP64, tol=tol)
    lat64 = []
    for _ in range(max(2, args.steps // 3)):
        s0 = time.perf_counter()
        r64 = ctx.solve(P.SOLVE_FP64, tol=tol)[0]
        lat64.append(time.perf_counter() - s0)
    u64 = ctx.gamma_values()
    rel_err = float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64))

    # Inputs starting in host memory: g at x* and f on the grid uploaded (set_rhs also forms
    # the particular solution on the device), the refined solve, u_gamma read back.  Context
    # set-up (point sets, closure, LGF table) is not repeated.  Reported beside `value`.
    g_host, f_host = p.g(xs), p.f_grid()
    host = []
    for _ in range(3):
        s0 = time.perf_counter()
        ctx.set_rhs(g_host, f_host)
        rh = ctx.solve(P.SOLVE_FP32_REFINED, tol=tol)[0]
        ctx.gamma_values()
        host.append(time.perf_counter() - s0)
    t_host = float(np.median(host))
    host_inclusive = {"ms_per_solve": t_host * 1e3,
                      "pair_interactions_per_s": (rh["matvecs_fp64"] + rh["matvecs_fp32"]) * pairs_mv / t_host,
                      "includes": "g (|gamma-| FP64) and f (n^3 FP64) uploaded from host memory, the particular "
                                  "solution, the refined solve, u_gamma read back"}
    log(f"fp64: {np.median(lat64) * 1e3:.1f} ms iters {r64['iterations']}; refined vs fp64 rel err {rel_err:.2e}")

    q = torch.from_numpy(np.random.default_rng(5).standard_normal(z["n_gamma_minus"])).to(dev)
    v = torch.empty(z["n_targets"], dtype=torch.float64, device=dev)
    mv, roof, ops = {}, {}, {}
    for name, prec in (("fp32", P.PREC_FP32), ("fp64", P.PREC_FP64)):
        t_med = time_applies(torch, ctx, q, v, prec, args.matvec_reps)
        t_sum = time_sum_kernel(torch, ctx, q, prec, max(3, args.matvec_reps // 4))
        st = ctx.sum_stats(prec)
        fl = flops_of(st, name)
        mv[name] = {"median_ms": t_med * 1e3, "pairs_per_s": pairs_mv / t_med, "sum_kernel_ms": t_sum * 1e3,
                    "tflops": fl / t_sum / 1e12, "tops": ops_of(st, name) / t_sum / 1e12, "pair_classes": st}
        roof[name] = fl / t_sum / 1e12
        ops[name] = ops_of(st, name) / t_sum / 1e12
    traffic = MEASURED_TRAFFIC["bytes"] if (kernel_hash() == MEASURED_TRAFFIC["sources_sha256_16"]
                                            and args.nodes == 129) else None
    # The sum is bound by VALU issue: table lookups replace most of the far-field flops
    # by integer index work, so the roofline counts lane-operations; the flop view follows.
    roofline = {"bound": "alu", "achieved": ops["fp32"], "peak": PEAK_VALU_OPS,
                "unit": "Top/s (VALU lane-operations, FMA = 1)", "frac": ops["fp32"] / PEAK_VALU_OPS,
                "traffic": traffic,
                "kernel": "lgf_sum_kernel<float,1> (HIP events around back-to-back launches of the sum alone)",
                "ops_per_launch": ops_of(mv["fp32"]["pair_classes"], "fp32"),
                "flops": {"achieved": roof["fp32"], "peak": PEAK_FP32_VECTOR, "unit": "TFLOP/s",
                          "frac": roof["fp32"] / PEAK_FP32_VECTOR,
                          "flops_per_launch": flops_of(mv["fp32"]["pair_classes"], "fp32")}}

    out = {
        "metric": METRIC,
        "value": pairs_total / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 LGF sum + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"poisson_ellipsoid_{args.nodes}^3",
                   "geometry": "ellipsoid (0.45,0.3,0.25) in unit cube", "h": p.h, "sigma": 0.0,
                   "gamma_targets": z["n_targets"], "sources": z["n_sources"], "pairs_per_matvec": pairs_mv,
                   "tol": tol},
        "solves_per_s": args.steps / elapsed,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "refined": {"iterations": refined["iterations"], "outer_steps": refined["outer_steps"],
                    "matvecs_fp32": refined["matvecs_fp32"], "matvecs_fp64": refined["matvecs_fp64"],
                    "rel_residual": refined["rel_residual_true"], "rel_err_vs_fp64_gpu": rel_err},
        "fp64_plain": {"solves_per_s": 1.0 / float(np.mean(lat64)), "p50_ms": float(np.percentile(lat64, 50) * 1e3),
                       "p99_ms": float(np.percentile(lat64, 99) * 1e3), "iterations": r64["iterations"],
                       "rel_residual": r64["rel_residual_true"]},
        "matvec": mv,
        "roofline": roofline,
        "fp64_sum": {"ops_frac": ops["fp64"] / PEAK_VALU_OPS, "flops_frac_of_fp64_peak": roof["fp64"] / PEAK_FP64_VECTOR},
        "setup_s": t_setup,
        "host_inclusive": host_inclusive,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    ctx.close()
    return out


def formulations(args, torch, P, W):
    """Single- against double-layer formulation (Sec. 3.4) on the 129^3 Poisson ellipsoid:
    iterations and solve time of each, FP64 and refined, and the difference of their u_gamma."""
    p = W.poisson_ellipsoid(args.nodes)
    out = {"workload": f"formulations_poisson_ellipsoid_{args.nodes}^3"}
    with P.Context.from_problem(p, max_krylov=400) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs), p.f_grid())
        ug = {}
        for lname, layer in (("double", P.LAYER_DOUBLE), ("single", P.LAYER_SINGLE)):
            for pname, prec in (("fp64", P.SOLVE_FP64), ("fp32_refined", P.SOLVE_FP32_REFINED)):
                ctx.solve(prec, tol=1e-10, formulation=layer)
                lat = []
                for _ in range(3):
                    s0 = time.perf_counter()
                    r = ctx.solve(prec, tol=1e-10, formulation=layer)[0]
                    lat.append(time.perf_counter() - s0)
                out[f"{lname}_{pname}"] = {"ms": float(np.median(lat) * 1e3), "iterations": r["iterations"],
                                           "outer_steps": r["outer_steps"], "converged": bool(r["converged"]),
                                           "rel_residual": r["rel_residual_true"]}
                ug[(lname, pname)] = ctx.gamma_values()
        ref = ug[("double", "fp64")]
        out["u_gamma_rel_diff_vs_double_fp64"] = {f"{k[0]}_{k[1]}": float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
                                                 for k, v in ug.items()}
    return out


def particular(args, torch, P, W):
    """Free-space volume potential against the finite-grid solve by sine transforms (Algorithm
    1) for u_p on the 129^3 Poisson ellipsoid: set_rhs time, and a refined solve with the grid
    solution, whose u_p on M+ is one more LGF sum (free) or a gather (box)."""
    p = W.poisson_ellipsoid(args.nodes)
    out = {"workload": f"particular_poisson_ellipsoid_{args.nodes}^3"}
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        g, f = p.g(xs), p.f_grid()
        u = {}
        for name in ("free", "box"):
            ctx.set_rhs(g, f, particular=name)
            ctx.solve(P.SOLVE_FP32_REFINED, tol=1e-10, compute_grid=True)
            t_rhs, t_solve = [], []
            for _ in range(3):
                s0 = time.perf_counter()
                ctx.set_rhs(g, f, particular=name)
                t_rhs.append(time.perf_counter() - s0)
                s0 = time.perf_counter()
                r = ctx.solve(P.SOLVE_FP32_REFINED, tol=1e-10, compute_grid=True)[0]
                t_solve.append(time.perf_counter() - s0)
            u[name] = ctx.solution()
            out[name] = {"set_rhs_ms": float(np.median(t_rhs) * 1e3),
                         "solve_with_grid_ms": float(np.median(t_solve) * 1e3), "iterations": r["iterations"]}
        m = ~np.isnan(u["free"])
        out["grid_solution_max_rel_diff"] = float(np.abs(u["box"][m] - u["free"][m]).max() / np.abs(u["free"][m]).max())
    return out


def laplace_sphere(args, torch, P, W):
    p = W.laplace_sphere()
    with P.Context.from_problem(p) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs))
        res = {}
        for name, prec in (("fp64", P.SOLVE_FP64), ("fp32_refined", P.SOLVE_FP32_REFINED)):
            for _ in range(args.warmup):
                ctx.solve(prec, tol=1e-10)
            lat = []
            for _ in range(max(args.steps, 10)):
                s0 = time.perf_counter()
                r = ctx.solve(prec, tol=1e-10)[0]
                lat.append(time.perf_counter() - s0)
            res[name] = {"solves_per_s": len(lat) / sum(lat), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                         "p99_ms": float(np.percentile(lat, 99) * 1e3), "iterations": r["iterations"],
                         "rel_residual": r["rel_residual_true"]}
        X = np.concatenate(ctx.sets()[:2]) * p.h
        err = np.abs(ctx.gamma_values() - p.exact(*X.T)).max()
        return {"workload": "laplace_sphere_33^3", "sizes": ctx.sizes, **res, "max_err_vs_exact": float(err)}


def helmholtz_star(args, torch, P, W):
    p = W.helmholtz_star(args.star_nodes)
    t0 = time.perf_counter()
    with P.Context.from_problem(p, max_rhs=16, max_krylov=200) as ctx:
        xs, _, _ = ctx.boundary_points()
        G = np.stack([p.g(xs, r) for r in range(16)])
        ctx.set_rhs(G)
        t_setup = time.perf_counter() - t0
        z = ctx.sizes
        pairs_mv = z["n_targets"] * z["n_sources"] * 16
        dev = torch.device("cuda:0")
        q = torch.from_numpy(np.random.default_rng(6).standard_normal((16, z["n_gamma_minus"]))).to(dev)
        v = torch.empty((16, z["n_targets"]), dtype=torch.float64, device=dev)
        mv = {}
        for name, prec in (("fp32", P.PREC_FP32), ("fp64", P.PREC_FP64)):
            t_med = time_applies(torch, ctx, q, v, prec, 5)
            mv[name] = {"median_ms": t_med * 1e3, "pair_rhs_per_s": pairs_mv / t_med}
            log(f"star 16-RHS matvec {name}: {t_med * 1e3:.1f} ms")
        s0 = time.perf_counter()
        res = ctx.solve(P.SOLVE_FP32_REFINED, tol=1e-10)
        t_solve = time.perf_counter() - s0
        log(f"star solve {t_solve:.2f}s iters {res[0]['iterations']}")
        return {"workload": f"helmholtz_star_{args.star_nodes}^3_16rhs", "sizes": z, "setup_s": t_setup,
                "matvec": mv, "solve_s": t_solve, "iterations": res[0]["iterations"],
                "outer_steps": res[0]["outer_steps"], "converged": all(r["converged"] for r in res),
                "max_rel_residual": max(r["rel_residual_true"] for r in res),
                "pair_rhs_per_s_in_solve": (res[0]["matvecs_fp32"] + res[0]["matvecs_fp64"]) * pairs_mv / t_solve}


def resolved_problems(P, count, make):
    """Seeded problems, redrawing those whose grid leaves a gamma- node with an empty D_n."""
    out, i = [], 0
    while len(out) < count:
        p = make(i)
        i += 1
        c = P.Context.from_problem(p, max_rhs=1, max_krylov=150)
        if c.sizes["n_empty_d"]:
            c.close()
            continue
        out.append((p, c))
    return out


def batch(args, torch, P, W):
    t0 = time.perf_counter()
    probs = resolved_problems(P, args.batch, W.batch_problem)
    for p, c in probs:
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
    t_setup = time.perf_counter() - t0
    ctxs = [c for _, c in probs]
    pairs = sum(c.sizes["n_targets"] * c.sizes["n_sources"] for c in ctxs)
    out = {"workload": f"batch_{len(ctxs)}", "setup_s": t_setup, "pairs_per_matvec_sum": pairs}
    with P.Batch(ctxs) as b:
        out["autotune"] = b.autotune(P.PREC_FP32)
        for name, prec in (("fp64", P.SOLVE_FP64), ("fp32_refined", P.SOLVE_FP32_REFINED)):
            b.solve(prec, tol=1e-10)                      # warm-up (captures the graph)
            s0 = time.perf_counter()
            res = b.solve(prec, tol=1e-10)
            dt = time.perf_counter() - s0
            out[name] = {"wall_s": dt, "solves_per_s": len(ctxs) / dt,
                         "converged": sum(r["converged"] for r in res),
                         "max_iterations": max(r["iterations"] for r in res),
                         "lockstep_matvecs": res[0]["matvecs_fp32"] + res[0]["matvecs_fp64"]}
            log(f"batch {name}: {dt:.2f}s for {len(ctxs)} solves")
    for c in ctxs:
        c.close()
    return out


def serve(args, torch, P, W):
    sizes = W.serving_stream(args.requests, 1.0)[1]
    probs = []
    i = 0
    while len(probs) < args.requests:
        p = W.serving_problem(i, int(sizes[len(probs)]))
        i += 1
        with P.Context.from_problem(p, max_rhs=1, max_krylov=200) as c:
            if c.sizes["n_empty_d"]:
                continue
        probs.append(p)
    budget = int(args.serve_budget_gb * (1 << 30))

    def run(rate):
        arrivals = W.serving_stream(args.requests, rate)[0] if rate else np.zeros(args.requests)
        with P.Server(hbm_budget=budget, max_slots=args.slots, precision=P.SOLVE_FP32_REFINED, tol=1e-10) as srv:
            t0 = time.perf_counter()
            tickets = []
            for a, p in zip(arrivals, probs):
                while time.perf_counter() - t0 < a:
                    time.sleep(0.0005)
                tickets.append(srv.submit_problem(p))
            lat = []
            for t in tickets:
                r, info, q, u = srv.result(t)
                lat.append(info["t_done"] - info["t_submit"])
            wall = time.perf_counter() - t0
            st = srv.stats()
        return {"rate": rate, "solves_per_s": len(probs) / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_active": st["max_active"],
                "peak_gb": st["peak_bytes"] / (1 << 30), "failed": st["failed"]}

    results = {"saturated": run(0.0)}
    log(f"serve saturated: {results['saturated']}")
    for f in (0.25, 0.5, 1.0, 2.0):
        r = run(f * results["saturated"]["solves_per_s"])
        results[f"x{f}"] = r
        log(f"serve rate x{f}: {r}")
    return {"workload": f"serve_{args.requests}_requests", "budget_gb": args.serve_budget_gb, "slots": args.slots,
            **results}


def profile(args, torch, P, W):
    """Matvecs only: FP32 then FP64 double-layer applies, then a 256 MiB device copy."""
    dev = torch.device("cuda:0")
    p = W.poisson_ellipsoid(args.nodes)
    with P.Context.from_problem(p) as ctx:
        z = ctx.sizes
        q = torch.from_numpy(np.random.default_rng(5).standard_normal(z["n_gamma_minus"])).to(dev)
        v = torch.empty(z["n_targets"], dtype=torch.float64, device=dev)
        for prec in (P.PREC_FP32, P.PREC_FP64):
            for _ in range(args.steps):
                ctx.apply_double_layer(q, v, prec)
        torch.cuda.synchronize()
    a = torch.empty(1 << 25, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"workload": "profile", "copy_bytes_each_way": a.numel() * 8}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nodes", type=int, default=129, help="nodes per axis of the ellipsoid (h = 1/(nodes-1))")
    ap.add_argument("--workload", default="poisson_ellipsoid",
                    choices=["poisson_ellipsoid", "laplace_sphere", "helmholtz_star", "batch", "serve", "profile",
                             "formulations", "particular"])
    ap.add_argument("--star-nodes", type=int, default=257)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2502_05507_amd as P
    import workloads as W

    fn = {"poisson_ellipsoid": headline, "laplace_sphere": laplace_sphere, "helmholtz_star": helmholtz_star,
          "formulations": formulations, "particular": particular,
          "batch": batch, "serve": serve, "profile": profile}[args.workload]
    print(json.dumps(fn(args, torch, P, W)))


if __name__ == "__main__":
    main()
