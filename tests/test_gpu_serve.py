"""Continuous batching on the GPU: every result is identical alone and in
the mix (each request has its own plan and workspace; same kernels, same
tiles), requests overlap, and the budget holds."""
import sys

import numpy as np
import pytest

from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch
    from paper_2208_14639_amd import vv10
    from paper_2208_14639_amd.serve import GpuExecutor, Request, Server
    rng = np.random.default_rng(5)
    pool = [inputs.make_problem(int(rng.integers(1, 4)), int(rng.integers(100, 400)), 500 + k)
            for k in range(5)]
    alone = []
    for p in pool:
        with vv10.Plan(p, prec="bf16x3", tiles="auto") as pl:
            e, _, _ = pl.energy_potential()
            H = pl.hessian_terms(p.rho_x, p.grad_rho_x)["hess"]
            torch.cuda.synchronize()
            alone.append((e.item(), H.cpu().numpy()))
    ex = GpuExecutor(prec="bf16x3", n_slots=3)
    budget = 3 * max(ex.footprint(p) for p in pool)
    srv = Server(ex, budget, n_slots=3)
    order = [0, 1, 2, 3, 4, 0, 2, 1, 3, 4, 0]
    futs = [srv.submit(Request(k, f"m{m}", pool[m]), at=0.0005 * k) for k, m in enumerate(order)]
    srv.run_until_idle(timeout_s=120)
    for k, m in enumerate(order):
        e, H = futs[k].result()
        assert e == alone[m][0]
        assert np.array_equal(H, alone[m][1])
    st = srv.stats()
    print("served stats", st, file=sys.stderr, flush=True)
    assert st["completed"] == len(order)
    assert srv.peak_used <= budget
    reqs = sorted(srv.done, key=lambda r: r.rid)
    assert any(b.admitted < a.finished and b.admitted > a.admitted for a in reqs for b in reqs)
    srv.close()
