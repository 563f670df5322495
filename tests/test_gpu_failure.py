"""A bounded wait of the LGF sum's work hand-off that gives up is reported as BAE_ERR_HIP,
never returned as a silently wrong result, and the context stays usable.  The give-up is
forced from the host (a context whose waits may poll zero times), so every kernel still
exits normally."""
import numpy as np
import pytest

import paper_2502_05507_amd as P

import workloads as W

from gpu_common import device, oracle_setup, rel_l2

pytestmark = pytest.mark.gpu


def test_give_up_is_reported_and_the_context_recovers():
    import torch
    dev = device()
    p = W.laplace_sphere(49)
    with P.Context.from_problem(p, sum_wait_polls=-1) as c:
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
        for prec in (P.SOLVE_FP64, P.SOLVE_FP32_REFINED):
            with pytest.raises(P.BaeError) as e:
                c.solve(prec, tol=1e-10)
            assert e.value.status == -5
        # an asynchronous apply: its failure is reported by the next call on the context
        q = torch.ones(c.sizes["n_gamma_minus"], dtype=torch.float64, device=dev)
        v = torch.empty(c.sizes["n_targets"], dtype=torch.float64, device=dev)
        c.apply_double_layer(q, v, P.PREC_FP32)
        torch.cuda.synchronize()
        with pytest.raises(P.BaeError) as e:
            c.apply_double_layer(q, v, P.PREC_FP32)
        assert e.value.status == -5
        torch.cuda.synchronize()
    # a context with the default bound on the same device solves correctly afterwards
    with P.Context.from_problem(p) as c:
        xs, _, _ = c.boundary_points()
        c.set_rhs(p.g(xs))
        r = c.solve(P.SOLVE_FP64, tol=1e-12)[0]
        assert r["converged"]
        g, G = oracle_setup(p)
        from oracle import operators
        q = torch.from_numpy(np.ones(c.sizes["n_gamma_minus"])).to(dev)
        v = torch.empty(c.sizes["n_targets"], dtype=torch.float64, device=dev)
        c.apply_double_layer(q, v, P.PREC_FP64)
        ref = operators.double_layer(g, G, np.ones(len(g.gamma_minus)), operators.gamma_targets(g))
        assert rel_l2(v.cpu().numpy(), ref) < 1e-10
