"""Shared helpers of the GPU tests: seeded inputs, the oracle side of each comparison."""
import numpy as np

import workloads as W
from oracle import geometry, lgf, operators


def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def small_problem(kind, n, sigma=0.0):
    h = 1.0 / (n - 1)
    params = {"sphere": (0.37,), "ellipsoid": (0.45, 0.3, 0.25), "torus": (0.28, 0.12),
              "star": (0.33, 0.15, 3.0, 2.0)}[kind]
    return W.Problem(f"{kind}{n}", (n, n, n), h, (0.0, 0.0, 0.0), float(sigma), kind, (0.5, 0.5, 0.5), params)


def oracle_setup(p):
    g = geometry.from_problem(p)
    G = lgf.LGFTable(g.max_offset(), p.sigma * p.h ** 2)
    return g, G


def rel_l2(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
