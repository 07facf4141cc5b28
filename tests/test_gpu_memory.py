"""The library's device-memory cache: freed plans' blocks are reused by the
next plans of similar size and returned on request."""
import pytest

from gpu_util import problem

pytestmark = pytest.mark.gpu


def test_plan_memory_is_cached_and_reused():
    import torch
    from paper_2208_14639_amd import vv10
    vv10.vv10_release_cached()
    assert vv10.vv10_cached_bytes() == 0
    p = problem(2, 200, 9)
    with vv10.Plan(p, prec="bf16x3") as pl:
        pl.hessian_terms(p.rho_x, p.grad_rho_x)
        torch.cuda.synchronize()
    held = vv10.vv10_cached_bytes()
    assert held > 0                      # the plan's blocks went to the cache
    with vv10.Plan(p, prec="bf16x3") as pl:
        H = pl.hessian_terms(p.rho_x, p.grad_rho_x)["hess"]
        torch.cuda.synchronize()
        assert vv10.vv10_cached_bytes() < held      # served from the cache
        assert torch.isfinite(H).all()
    vv10.vv10_release_cached()
    assert vv10.vv10_cached_bytes() == 0
