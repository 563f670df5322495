#!/usr/bin/env python3
"""Benchmark of the unfitted-BAE hot path on one MI355X.

Default workload (the JSON line the contract asks for; the largest single-GPU
configuration): modified Helmholtz -Lap u + kappa^2 u = 0, kappa^2 = 10, on the star
r = 0.4 (1 + 0.15 sin 3 theta cos 2 phi) centred in the unit cube, h = 1/256 (257^3 nodes),
16 right-hand sides (seeded harmonic-polynomial boundary data).  One step = one complete
Algorithm 1 solve of all 16 right-hand sides on device-resident inputs: the right-hand side
(bae_set_rhs_device), then FP64 iterative refinement around GMRES whose matvecs run the FP32
16-RHS LGF sum on the matrix cores (every matvec = double-layer weights, the LGF sum over
|gamma| x |gamma- u E| pairs for 16 densities, the closure), the FP64 residual matvecs, the
last of which gives u_gamma.  value = LGF pair-interactions (pairs x right-hand sides)
evaluated in the timed steps divided by their wall time.  Also reported: solves/s (one per
right-hand side) and p50/p99 step latency of the refined path and of the plain FP64 path,
the roofline of the dominant kernel (the FP32 16-RHS matrix-core sum: algorithmic flops per
launch over its own duration, HIP events around back-to-back launches of the sum alone, on
the stream it runs on), and the CPU oracle on 2,000 seeded rows of the same matvec, on one
core and on all cores.  The 129^3 Poisson ellipsoid (the one-RHS VALU sum) is reported
beside it under "poisson_ellipsoid_129".

Other workloads (--workload; their own JSON line, not the contract's):
  poisson_ellipsoid  129^3 Poisson ellipsoid, one RHS, FP32 VALU sum (the former headline)
  laplace_sphere     33^3 Laplace sphere, FP64 and refined solve latency, the oracle's solve rate
  batch              512 seeded small problems in one lock-step, graph-replayed batch
  serve              Poisson arrivals into the continuous-batching server, p50/p99 latency
  profile            129^3 matvecs only (for rocprofv3) plus a device copy of known size
  profile_star       257^3 16-RHS FP32 sums only (for rocprofv3) plus the same copy
  profile_fft        FFT-convolution matvecs only (129^3 ellipsoid, 257^3 star) plus the same copy
  profile_box        the box particular solution alone at --nodes per axis plus the same copy
  formulations       single- against double-layer formulation (iterations, time) at 129^3
  particular         free-space against finite-grid (sine-transform) particular solution at 129^3
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LGF pair-interactions/s per BAE matvec; solves/s + p99 latency at rel err ≤1e-8"
PEAK_FP32 = 157.3   # TFLOP/s, MI355X published FP32 peak (vector and matrix cores)
PEAK_FP64 = 78.6    # TFLOP/s
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per second
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic flop convention (frozen with the oracle's far-field formula): a far-field
# kernel value costs 32 flop (the corrected q = 3 expansion: 3 differences, 3 squares, 2 adds,
# e2 4, e3 1, rsqrt 1, rho 1, x and y 4, the degree-8 polynomial 6, the degree-4 term 2, the
# bracket 4, the final product 1); every (pair, right-hand side) adds its multiply-accumulate,
# 2 flop.  Table lookups and global-table gathers generate their value without flops.
# Compensation and index arithmetic are overhead, not counted.
F_FAR = 32
F_RHS = 2


def kernel_hash(files=("paper_2502_05507_amd/csrc/lgf_sum.hip", "paper_2502_05507_amd/csrc/lgf_device.hpp")):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


# Counter measurements of the dominant kernels (rocprofv3 --pmc runs of `bench.py --workload
# profile_star` / `profile`, profiles/*_counters.md), valid only for the kernel sources they
# were taken on (their hash): HBM bytes per launch (FETCH_SIZE x f + WRITE_SIZE x w, the
# factors calibrated on copies of known size), VALU-issue and matrix-core-busy shares.
MEASURED = {
    "lgf_sum_mfma_helmholtz_star_257": {"sources_sha256_16": "211868e5dbd39cd9",
                                        "bytes": (1.3422e7 * 2.0 + 1.0688e6 * 1.0) * 1024,
                                        "valu_issue": 0.765, "valu_busy": 0.823, "mfma_busy": 0.264,
                                        "l2_hit": 0.697},
    "lgf_sum_poisson_ellipsoid_129": {"sources_sha256_16": "211868e5dbd39cd9",
                                      "bytes": (12283 * 2.0 + 18519 * 1.0) * 1024,
                                      "valu_issue": 0.872},
}


def measured(key):
    m = MEASURED.get(key)
    return m if m and m["sources_sha256_16"] == kernel_hash() else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def far_values(stats, prec, sigma0, far_ok):
    """Kernel values of one launch that the far-field expansion generates (bae_sum_stats
    classes): the FP32 far blocks, the FP64 far blocks at sigma = 0, and the far part of mixed
    blocks when the sum has a far field."""
    v = stats["far_q2"]
    if prec == "fp64" and sigma0:
        v += stats["far"]
    if far_ok:
        v += stats["mixed_far"]
    return v


def flops_of(stats, prec, nrhs, sigma0, far_ok):
    """Algorithmic flops of one launch of the LGF sum (F_FAR per far-field value, F_RHS per
    pair and right-hand side)."""
    pairs = sum(stats.values())
    return F_FAR * far_values(stats, prec, sigma0, far_ok) + F_RHS * nrhs * pairs


PEAK_HBM = 8000.0   # GB/s, MI355X HBM3E


def conv_bytes(z):
    """Algorithmic HBM bytes of one FFT convolution (one right-hand side) on the box of extents
    e with FFT lengths M (bae_sizes conv_box / conv_fft): every pass reads and writes the pruned
    arrays once -- real box E, half-spectrum rows e0 e1 H2, planes e0 M1 H2, the kernel's
    transform on one octant H0 H1 H2 (complex 16 B, real 8 B)."""
    e, M = z["conv_box"], z["conv_fft"]
    H = [m // 2 + 1 for m in M]
    E = e[0] * e[1] * e[2]
    rows = e[0] * e[1] * H[2]
    planes = e[0] * M[1] * H[2]
    return (8 * E + 16 * rows) + (16 * rows + 16 * planes) + (32 * planes + 8 * H[0] * H[1] * H[2]) \
        + (16 * planes + 16 * rows) + (16 * rows + 8 * E)


def fast_summation(torch, P, ctx, step_fft, steps, z, nrhs, q, ref_u, log_name):
    """The FFT-convolution path on the same context: solves (every matvec a convolution, FP64),
    the convolution alone, and its HBM roofline."""
    step_fft()
    lat, pairs_total = [], 0
    pairs_mv = z["n_targets"] * z["n_sources"] * nrhs
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        res = step_fft()
        lat.append(time.perf_counter() - s0)
        pairs_total += (res[0]["matvecs_fp64"] + res[0]["matvecs_fp32"]) * pairs_mv
    elapsed = time.perf_counter() - t0
    u = np.stack([ctx.gamma_values(r) for r in range(nrhs)])
    err = float(max(np.linalg.norm(u[r] - ref_u[r]) / np.linalg.norm(ref_u[r]) for r in range(nrhs)))
    t_conv = time_sum_kernel(torch, ctx, q, P.PREC_FFT, 3, burst=3) / nrhs
    zz = ctx.get_sizes()
    b = conv_bytes(zz)
    log(f"{log_name} fft: {np.median(lat) * 1e3:.0f} ms per step, convolution {t_conv * 1e3:.3f} ms per RHS")
    return {"pair_interactions_per_s": pairs_total / elapsed, "solves_per_s": nrhs * steps / elapsed,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "iterations": max(r["iterations"] for r in res), "max_rel_residual": max(r["rel_residual_true"] for r in res),
            "max_rel_diff_vs_headline_path": err,
            "convolution_ms_per_rhs": t_conv * 1e3, "matvec_pair_interactions_per_s": pairs_mv / (t_conv * nrhs),
            "box": zz["conv_box"], "fft_lengths": zz["conv_fft"],
            "roofline": {"bound": "hbm", "achieved": b / t_conv / 1e9, "peak": PEAK_HBM, "unit": "GB/s",
                         "frac": b / t_conv / 1e9 / PEAK_HBM, "bytes_per_convolution": b,
                         "kernel": "one convolution (HIP events): clear, scatter of the weights, the five FFT passes (conv_z_fwd, conv_lines x3, conv_z_inv), gather; bytes count the FFT passes"}}


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
    """Average duration of the LGF-sum kernel alone: HIP events on the launch stream (torch's
    current stream, which the library launches on) around 1 and 1 + burst back-to-back
    launches (bae_lgf_sum_repeat, which forms the weights once first); the difference over
    burst removes the weights launch and the event overhead."""
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


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Cores this process may use, capped at the 16 a one-GPU machine grants."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# ----------------------------------------------------------------------------- CPU oracle
_ORACLE = {}


def _oracle_rows(task):
    """Worker: the oracle's literal double-layer sum at a block of target rows, one density."""
    from oracle import operators
    rows, r = task
    geo, G, Q = _ORACLE["geo"], _ORACLE["G"], _ORACLE["Q"]
    return operators.double_layer(geo, G, Q[r], rows)


def cpu_baseline_worker(workload, nrows, nrhs_all):
    """Runs in a child process that never touches the GPU: the oracle (plain FP64 NumPy) on
    `nrows` seeded target rows of the workload's matvec -- one density on one core, then
    `nrhs_all` densities over every core (a fork pool).  Prints one JSON object."""
    import multiprocessing as mp
    import workloads as W
    from oracle import geometry, lgf, operators
    p = {"helmholtz_star": lambda: W.helmholtz_star(257), "poisson_ellipsoid": lambda: W.poisson_ellipsoid(129)}[workload]()
    t0 = time.perf_counter()
    geo = geometry.from_problem(p)
    G = lgf.LGFTable(geo.max_offset(), p.sigma * p.h ** 2)
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(2000)
    T = operators.gamma_targets(geo)
    rows = T[np.sort(rng.choice(len(T), size=min(nrows, len(T)), replace=False))]
    cores = host_cores()
    nrhs_all = nrhs_all if nrhs_all > 0 else cores
    Q = rng.standard_normal((nrhs_all, len(geo.gamma_minus)))
    n_src = len(geo.gamma_minus) + len(geo.ext)
    _ORACLE.update(geo=geo, G=G, Q=Q)
    blocks = [rows[i:i + 32] for i in range(0, len(rows), 32)]
    t0 = time.perf_counter()
    for b in blocks:
        _oracle_rows((b, 0))
    t1 = time.perf_counter() - t0
    tasks = [(b, r) for r in range(nrhs_all) for b in blocks]
    with mp.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_rows, tasks, chunksize=max(1, len(tasks) // (4 * cores)))
        tall = time.perf_counter() - t0
    print(json.dumps({"single": len(rows) * n_src / t1, "all": len(rows) * n_src * nrhs_all / tall, "nrhs": nrhs_all,
                      "t_single": t1, "t_all": tall, "rows": len(rows), "targets": len(T), "sources": n_src,
                      "cores": cores, "setup_s": t_setup}))


def cpu_baseline(workload, nrows, nrhs_all):
    """The oracle timed on this machine's host cores, in a child process (the benchmark's own
    process holds the GPU), on a bounded sample of the workload's matvec."""
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", workload,
                          "--cpu-rows", str(nrows), "--cpu-rhs", str(nrhs_all)],
                         capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(f"cpu baseline worker failed: {out.stderr[-2000:]}")
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["all"], "unit": "pair-interactions/s", "cores": r["cores"], "kind": "oracle",
            "sample": f"{r['rows']} seeded of {r['targets']} gamma target rows x {r['sources']} sources x "
                      f"{r['nrhs']} densities (literal double-layer sum, FP64 NumPy) on {r['cores']} processes: "
                      f"{r['t_all']:.1f} s; one density on one core: {r['t_single']:.1f} s",
            "single_core_value": r["single"], "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def _oracle_solve_batch_problem(i):
    """Worker: the oracle's solve (its literal sums, its own GMRES) of batch problem i."""
    import workloads as W
    from oracle import bae as obae
    t0 = time.perf_counter()
    r = obae.solve(W.batch_problem(i))
    return {"i": i, "seconds": time.perf_counter() - t0, "iterations": len(r["history"]),
            "converged": bool(r["converged"])}


def oracle_batch_worker(indices):
    """Runs in a child process that never touches the GPU: the oracle's solves of the given
    batch problems, one per process over the host's cores.  Prints one JSON object."""
    import multiprocessing as mp
    cores = host_cores()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(cores, len(indices))) as pool:
        res = pool.map(_oracle_solve_batch_problem, indices, chunksize=1)
    print(json.dumps({"wall_s": time.perf_counter() - t0, "cores": cores, "solves": res}))


def oracle_batch_sample(probs, results, count=16):
    """The oracle's solves of a seeded sample of the batch, the first `count` problems of the
    stream (one per host core; the largest takes the oracle about a minute), timed in a child
    process; with the batch's own pair and iteration counts, an estimate of the oracle's time
    for the whole batch."""
    pick = list(range(min(count, len(probs))))
    idx = [int(probs[k][0].name[len("batch"):]) for k in pick]
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-batch-worker",
                          ",".join(str(i) for i in idx)], capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(f"oracle batch worker failed: {out.stderr[-2000:]}")
    r = json.loads(out.stdout.strip().splitlines()[-1])
    work = lambda k, it: probs[k][1].sizes["n_targets"] * probs[k][1].sizes["n_sources"] * (it + 2)
    sample_work = sum(work(k, s["iterations"]) for k, s in zip(pick, r["solves"]))
    cpu_s = sum(s["seconds"] for s in r["solves"])
    batch_work = sum(work(k, res["iterations"]) for k, res in enumerate(results))
    return {"sample": f"the first {len(idx)} problems of the seeded stream",
            "problems": idx, "solves_per_s_all_cores": len(idx) / r["wall_s"], "wall_s": r["wall_s"],
            "cores": r["cores"], "cpu_s_per_solve": cpu_s / len(idx),
            "converged": sum(s["converged"] for s in r["solves"]),
            "batch_estimate_all_cores_s": batch_work * cpu_s / sample_work / r["cores"],
            "estimate": "(pairs per matvec) x (GMRES iterations + 2) over the batch, at the sample's oracle "
                        "seconds per pair-matvec, divided over the cores", "cpu_model": cpu_model()}


# ----------------------------------------------------------------------------- headline (257^3 star)
def headline(args, torch, P, W):
    dev = torch.device("cuda:0")
    nrhs = 16
    p = W.helmholtz_star(args.star_nodes)
    t_setup = time.perf_counter()
    ctx = P.Context.from_problem(p, max_rhs=nrhs, max_krylov=200)
    xs, _, _ = ctx.boundary_points()
    G = torch.from_numpy(np.stack([p.g(xs, r) for r in range(nrhs)])).to(dev)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    z = ctx.sizes
    pairs_mv = z["n_targets"] * z["n_sources"] * nrhs
    log(f"setup {t_setup:.2f}s sizes {z}")

    tol = 1e-10

    def step(prec):
        ctx.set_rhs_device(G)
        return ctx.solve(prec, tol=tol)

    for _ in range(args.warmup):
        step(P.SOLVE_FP32_REFINED)
    torch.cuda.synchronize()
    lat, pairs_total = [], 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        res = step(P.SOLVE_FP32_REFINED)
        lat.append(time.perf_counter() - s0)
        pairs_total += (res[0]["matvecs_fp64"] + res[0]["matvecs_fp32"]) * pairs_mv
        log(f"step {k}: {lat[-1] * 1e3:.0f} ms, iters {max(r['iterations'] for r in res)}, "
            f"outer {res[0]['outer_steps']}, relres {max(r['rel_residual_true'] for r in res):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    refined = res
    u32 = np.stack([ctx.gamma_values(r) for r in range(nrhs)])

    lat64 = []
    for _ in range(args.fp64_steps):
        s0 = time.perf_counter()
        r64 = step(P.SOLVE_FP64)
        lat64.append(time.perf_counter() - s0)
    u64 = np.stack([ctx.gamma_values(r) for r in range(nrhs)])
    rel_err = float(max(np.linalg.norm(u32[r] - u64[r]) / np.linalg.norm(u64[r]) for r in range(nrhs)))
    log(f"fp64: {np.median(lat64) * 1e3:.0f} ms iters {max(r['iterations'] for r in r64)}; "
        f"refined vs fp64 rel err {rel_err:.2e}")

    # the dominant kernel: the FP32 16-RHS matrix-core sum, alone
    q = torch.from_numpy(np.random.default_rng(6).standard_normal((nrhs, z["n_gamma_minus"]))).to(dev)
    t_sum = time_sum_kernel(torch, ctx, q, P.PREC_FP32, 3, burst=5)
    st32 = ctx.sum_stats(P.PREC_FP32)
    far_ok = bool(z["far_field_fp32"])
    fl = flops_of(st32, "fp32", nrhs, False, far_ok)
    t_sum64 = time_sum_kernel(torch, ctx, q, P.PREC_FP64, 2, burst=3)
    st64 = ctx.sum_stats(P.PREC_FP64)
    fl64 = flops_of(st64, "fp64", nrhs, False, bool(z["far_field_fp64"]))
    log(f"sum kernels: fp32 {t_sum * 1e3:.1f} ms, fp64 {t_sum64 * 1e3:.1f} ms")
    meas = measured("lgf_sum_mfma_helmholtz_star_257")
    roofline = {"bound": "mfma", "achieved": fl / t_sum / 1e12, "peak": PEAK_FP32, "unit": "TFLOP/s",
                "frac": fl / t_sum / 1e12 / PEAK_FP32, "traffic": meas["bytes"] if meas else None,
                "kernel": "lgf_sum_mfma_kernel<float> (FP32, 16 right-hand sides; HIP events around back-to-back "
                          "launches of the sum alone)",
                "kernel_ms": t_sum * 1e3, "flops_per_launch": fl,
                "flop_convention": f"{F_FAR} per far-field kernel value + {F_RHS} per (pair, RHS)",
                "pair_classes": st32,
                "valu_issue_share": meas["valu_issue"] if meas else None,
                "valu_busy_share": meas["valu_busy"] if meas else None,
                "mfma_busy_share": meas["mfma_busy"] if meas else None,
                "l2_hit_rate": meas["l2_hit"] if meas else None}

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
        "dtype": "f32 (16-RHS matrix-core LGF sum) + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"helmholtz_star_{args.star_nodes}^3_16rhs",
                   "geometry": "star r=0.4(1+0.15 sin3t cos2p) in unit cube", "h": p.h, "kappa2": p.sigma,
                   "rhs": nrhs, "gamma_targets": z["n_targets"], "sources": z["n_sources"],
                   "pairs_per_matvec": pairs_mv, "tol": tol},
        "solves_per_s": nrhs * args.steps / elapsed,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "latency_unit": "one step: set_rhs_device + refined solve of all 16 right-hand sides",
        "refined": {"iterations": max(r["iterations"] for r in refined), "outer_steps": refined[0]["outer_steps"],
                    "matvecs_fp32": refined[0]["matvecs_fp32"], "matvecs_fp64": refined[0]["matvecs_fp64"],
                    "max_rel_residual": max(r["rel_residual_true"] for r in refined),
                    "max_rel_err_vs_fp64_gpu": rel_err},
        "fp64_plain": {"solves_per_s": nrhs / float(np.mean(lat64)), "p50_ms": float(np.percentile(lat64, 50) * 1e3),
                       "p99_ms": float(np.percentile(lat64, 99) * 1e3),
                       "iterations": max(r["iterations"] for r in r64),
                       "max_rel_residual": max(r["rel_residual_true"] for r in r64)},
        "roofline": roofline,
        "fp64_sum": {"kernel_ms": t_sum64 * 1e3, "tflops": fl64 / t_sum64 / 1e12,
                     "frac_of_fp64_peak": fl64 / t_sum64 / 1e12 / PEAK_FP64, "pair_classes": st64},
        "setup_s": t_setup,
    }
    out["fast_summation"] = fast_summation(torch, P, ctx, lambda: step(P.SOLVE_FFT), max(1, min(args.steps, 3)), z,
                                           nrhs, q, u32, "star")
    ctx.close()
    if not args.no_extra:
        out["poisson_ellipsoid_129"] = ellipsoid(args, torch, P, W, steps=5, warmup=2, extra=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline("helmholtz_star", args.cpu_rows, args.cpu_rhs)
    return out


def ellipsoid(args, torch, P, W, steps=None, warmup=None, extra=False):
    """129^3 Poisson ellipsoid, one RHS: a step is set_rhs_box (f and g device-resident; the
    particular solution by sine transforms) + the refined solve."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    dev = torch.device("cuda:0")
    p = W.poisson_ellipsoid(args.nodes)
    t_setup = time.perf_counter()
    ctx = P.Context.from_problem(p)
    xs, _, _ = ctx.boundary_points()
    g = torch.from_numpy(p.g(xs)).to(dev)
    f = torch.from_numpy(p.f_grid()).to(dev)
    ctx.set_rhs_device(g, f, particular="box")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    z = ctx.sizes
    pairs_mv = z["n_targets"] * z["n_sources"]
    tol = 1e-10

    def step(prec):
        ctx.set_rhs_device(g, f, particular="box")
        return ctx.solve(prec, tol=tol)[0]

    for _ in range(warmup):
        step(P.SOLVE_FP32_REFINED)
    torch.cuda.synchronize()
    lat, pairs_total = [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        r = step(P.SOLVE_FP32_REFINED)
        lat.append(time.perf_counter() - s0)
        pairs_total += (r["matvecs_fp64"] + r["matvecs_fp32"]) * pairs_mv
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    u32 = ctx.gamma_values()
    lat64 = []
    for _ in range(max(2, steps // 3)):
        s0 = time.perf_counter()
        r64 = step(P.SOLVE_FP64)
        lat64.append(time.perf_counter() - s0)
    u64 = ctx.gamma_values()
    rel_err = float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64))
    q = torch.from_numpy(np.random.default_rng(5).standard_normal(z["n_gamma_minus"])).to(dev)
    v = torch.empty(z["n_targets"], dtype=torch.float64, device=dev)
    mv = {}
    for name, prec in (("fp32", P.PREC_FP32), ("fp64", P.PREC_FP64)):
        t_med = time_applies(torch, ctx, q, v, prec, args.matvec_reps)
        t_sum = time_sum_kernel(torch, ctx, q, prec, max(3, args.matvec_reps // 4))
        st = ctx.sum_stats(prec)
        fl = flops_of(st, name, 1, True, True)
        mv[name] = {"median_ms": t_med * 1e3, "pairs_per_s": pairs_mv / t_med, "sum_kernel_ms": t_sum * 1e3,
                    "tflops": fl / t_sum / 1e12,
                    "frac": fl / t_sum / 1e12 / (PEAK_FP32 if name == "fp32" else PEAK_FP64), "pair_classes": st}
    fast = fast_summation(torch, P, ctx, lambda: [step(P.SOLVE_FFT)], max(2, steps), z, 1, q, u32[None],
                          "ellipsoid")
    meas = measured("lgf_sum_poisson_ellipsoid_129")
    roofline = {"bound": "alu", "achieved": mv["fp32"]["tflops"], "peak": PEAK_FP32, "unit": "TFLOP/s",
                "frac": mv["fp32"]["frac"], "traffic": meas["bytes"] if meas else None,
                "kernel": "lgf_sum_kernel<float,1> (HIP events around back-to-back launches of the sum alone)",
                "flop_convention": f"{F_FAR} per far-field kernel value + {F_RHS} per pair",
                "valu_issue_share": meas["valu_issue"] if meas else None}
    ctx.close()
    body = {"config": {"workload": f"poisson_ellipsoid_{args.nodes}^3", "h": p.h, "sigma": 0.0,
                       "gamma_targets": z["n_targets"], "sources": z["n_sources"], "pairs_per_matvec": pairs_mv,
                       "tol": tol},
            "value": pairs_total / elapsed, "unit": "pair-interactions/s",
            "ms_per_step": elapsed / steps * 1e3, "solves_per_s": steps / elapsed,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "latency_unit": "one step: set_rhs_device (box particular solution) + refined solve",
            "refined": {"iterations": r["iterations"], "outer_steps": r["outer_steps"],
                        "matvecs_fp32": r["matvecs_fp32"], "matvecs_fp64": r["matvecs_fp64"],
                        "rel_residual": r["rel_residual_true"], "rel_err_vs_fp64_gpu": rel_err},
            "fp64_plain": {"solves_per_s": 1.0 / float(np.mean(lat64)),
                           "p50_ms": float(np.percentile(lat64, 50) * 1e3),
                           "p99_ms": float(np.percentile(lat64, 99) * 1e3), "iterations": r64["iterations"]},
            "matvec": mv, "roofline": roofline, "fast_summation": fast, "setup_s": t_setup}
    if extra:
        return body
    out = {"metric": METRIC, "value": body.pop("value"), "unit": body.pop("unit"), "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": body.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 LGF sum + f64 refinement", "data": "synthetic",
           "config": body.pop("config"), **body}
    if not args.no_cpu_baseline:
        cb = cpu_baseline("poisson_ellipsoid", args.cpu_rows, args.cpu_rhs)
        # a full oracle solve here takes about 10^11 pair evaluations: derived from the measured
        # matvec rate, not run
        n_mv = out["fp64_plain"]["iterations"] + 2
        cb["oracle_solve_estimate"] = {"matvecs": n_mv, "seconds_one_core": n_mv * pairs_mv / cb["single_core_value"],
                                       "seconds_all_cores": n_mv * pairs_mv / cb["value"],
                                       "solves_per_s_all_cores": cb["value"] / (n_mv * pairs_mv),
                                       "derived": "GMRES iterations of the FP64 GPU solve + 2 (true residual, "
                                                  "u_gamma) literal matvecs at the rates measured above; the "
                                                  "volume potential of f is not included"}
        out["cpu_baseline"] = cb
    return out


def formulations(args, torch, P, W):
    """Double-layer, single-layer (Sec. 3.4) and direct (Sec. 3.1) formulations on the 129^3
    Poisson ellipsoid: iterations and solve time of each, FP64 and refined, and the difference
    of their u_gamma."""
    p = W.poisson_ellipsoid(args.nodes)
    out = {"workload": f"formulations_poisson_ellipsoid_{args.nodes}^3"}
    with P.Context.from_problem(p, max_krylov=400) as ctx:
        xs, _, _ = ctx.boundary_points()
        ctx.set_rhs(p.g(xs), p.f_grid())
        ug = {}
        for lname, layer in (("double", P.LAYER_DOUBLE), ("single", P.LAYER_SINGLE), ("direct", P.LAYER_DIRECT)):
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
        ug = ctx.gamma_values()
        err = np.abs(ug - p.exact(*X.T)).max()
    out = {"workload": "laplace_sphere_33^3", "sizes": ctx.sizes, **res, "max_err_vs_exact": float(err)}
    if not args.no_cpu_baseline:
        # the oracle's solve of the same problem (its literal sums, its own GMRES), one process
        import resource
        from oracle import bae as obae
        c0 = resource.getrusage(resource.RUSAGE_SELF)
        t0 = time.perf_counter()
        ref = obae.solve(p, tol=1e-10)
        t_or = time.perf_counter() - t0
        c1 = resource.getrusage(resource.RUSAGE_SELF)
        cpu_s = (c1.ru_utime - c0.ru_utime) + (c1.ru_stime - c0.ru_stime)
        out["oracle_solve"] = {"solves_per_s": 1.0 / t_or, "seconds": t_or, "iterations": len(ref["history"]),
                               "u_gamma_rel_diff_vs_gpu": float(np.linalg.norm(ug - ref["u_gamma"]) /
                                                                np.linalg.norm(ref["u_gamma"])),
                               "cpu_seconds_per_wall_second": cpu_s / t_or, "cpu_model": cpu_model()}
    return out


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
    res64 = None
    with P.Batch(ctxs) as b:
        out["autotune"] = b.autotune(P.PREC_FP32)
        for name, prec in (("fp64", P.SOLVE_FP64), ("fp32_refined", P.SOLVE_FP32_REFINED)):
            b.solve(prec, tol=1e-10)                      # warm-up (captures the graph)
            s0 = time.perf_counter()
            res = b.solve(prec, tol=1e-10)
            dt = time.perf_counter() - s0
            if prec == P.SOLVE_FP64:
                res64 = res
            out[name] = {"wall_s": dt, "solves_per_s": len(ctxs) / dt,
                         "converged": sum(r["converged"] for r in res),
                         "max_iterations": max(r["iterations"] for r in res),
                         "lockstep_matvecs": res[0]["matvecs_fp32"] + res[0]["matvecs_fp64"]}
            log(f"batch {name}: {dt:.2f}s for {len(ctxs)} solves")
    if not args.no_cpu_baseline:
        out["oracle_sample"] = oracle_batch_sample(probs, res64)
        log(f"batch oracle sample: {out['oracle_sample']['solves_per_s_all_cores']:.3f} solves/s")
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


def profile_star(args, torch, P, W):
    """The 257^3 star's 16-RHS sums only: FP32 (matrix cores) then FP64 LGF-sum launches, then
    the same 256 MiB device copy (the counter runs' calibration)."""
    dev = torch.device("cuda:0")
    p = W.helmholtz_star(args.star_nodes)
    with P.Context.from_problem(p, max_rhs=16, max_krylov=8) as ctx:
        z = ctx.sizes
        q = torch.from_numpy(np.random.default_rng(6).standard_normal((16, z["n_gamma_minus"]))).to(dev)
        for prec in (P.PREC_FP32, P.PREC_FP64):
            ctx.lgf_sum_repeat(q, args.steps, prec)
            torch.cuda.synchronize()
            log(f"profile_star: {args.steps} sums done ({'fp32' if prec == P.PREC_FP32 else 'fp64'})")
    a = torch.empty(1 << 25, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"workload": "profile_star", "copy_bytes_each_way": a.numel() * 8, "sizes": z}


def profile_fft(args, torch, P, W):
    """FFT-convolution matvecs only (129^3 ellipsoid, then one right-hand side of the 257^3
    star), then the same 256 MiB device copy (the counter runs' calibration)."""
    dev = torch.device("cuda:0")
    for p, name in ((W.poisson_ellipsoid(args.nodes), "ellipsoid"), (W.helmholtz_star(args.star_nodes), "star")):
        with P.Context.from_problem(p, max_rhs=1, max_krylov=8) as ctx:
            z = ctx.sizes
            q = torch.from_numpy(np.random.default_rng(5).standard_normal(z["n_gamma_minus"])).to(dev)
            v = torch.empty(z["n_targets"], dtype=torch.float64, device=dev)
            for _ in range(args.steps):
                ctx.apply_double_layer(q, v, P.PREC_FFT)
            torch.cuda.synchronize()
            log(f"profile_fft: {args.steps} convolutions done ({name})")
    a = torch.empty(1 << 25, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"workload": "profile_fft", "copy_bytes_each_way": a.numel() * 8}


def profile_box(args, torch, P, W):
    """Algorithm 1's box particular solution alone (set_rhs_device with f on the device, the
    sine transforms by the LDS FFT) on the Poisson ellipsoid at --nodes per axis, then the same
    256 MiB device copy."""
    dev = torch.device("cuda:0")
    p = W.poisson_ellipsoid(args.nodes)
    with P.Context.from_problem(p, max_rhs=1, max_krylov=8) as ctx:
        xs, _, _ = ctx.boundary_points()
        g = torch.from_numpy(p.g(xs)).to(dev)
        f = torch.from_numpy(p.f_grid()).to(dev)
        for _ in range(args.steps):
            ctx.set_rhs_device(g, f, particular="box")
        torch.cuda.synchronize()
        log(f"profile_box: {args.steps} box solves done ({args.nodes}^3)")
    a = torch.empty(1 << 25, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"workload": f"profile_box_{args.nodes}^3", "copy_bytes_each_way": a.numel() * 8}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nodes", type=int, default=129, help="nodes per axis of the ellipsoid (h = 1/(nodes-1))")
    ap.add_argument("--workload", default="helmholtz_star",
                    choices=["helmholtz_star", "poisson_ellipsoid", "laplace_sphere", "batch", "serve", "profile",
                             "profile_star", "profile_fft", "profile_box", "formulations", "particular"])
    ap.add_argument("--star-nodes", type=int, default=257)
    ap.add_argument("--fp64-steps", type=int, default=1, help="plain FP64 solves timed beside the headline")
    ap.add_argument("--no-extra", action="store_true", help="skip the 129^3 ellipsoid beside the headline")
    ap.add_argument("--cpu-rows", type=int, default=2000, help="target rows of the CPU oracle sample")
    ap.add_argument("--cpu-rhs", type=int, default=1, help="densities of the all-core sample (0: one per core)")
    ap.add_argument("--cpu-baseline-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-batch-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=20)
    args = ap.parse_args()
    if args.cpu_baseline_worker:        # child process of cpu_baseline: CPU only
        cpu_baseline_worker(args.cpu_baseline_worker, args.cpu_rows, args.cpu_rhs)
        return
    if args.oracle_batch_worker:        # child process of oracle_batch_sample: CPU only
        oracle_batch_worker([int(v) for v in args.oracle_batch_worker.split(",")])
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2502_05507_amd as P
    import workloads as W

    fn = {"helmholtz_star": headline, "poisson_ellipsoid": ellipsoid, "laplace_sphere": laplace_sphere,
          "formulations": formulations, "particular": particular, "batch": batch, "serve": serve,
          "profile": profile, "profile_star": profile_star, "profile_fft": profile_fft,
          "profile_box": profile_box}[args.workload]
    print(json.dumps(fn(args, torch, P, W)))


if __name__ == "__main__":
    main()
