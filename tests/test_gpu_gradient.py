"""vv10_gradient -- the VV10 nuclear gradient alone (Section II.A) --
against the FP64 oracle and the gradient output of vv10_hessian_terms."""
import functools
import sys

import pytest

import oracle
from gpu_util import normwise, problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
V_NORM = 1e-5
CASES = [(1, 8, 11), (2, 37, 5), (2, 700, 1001), (6, 1500, 1002)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@functools.lru_cache(maxsize=8)
def oracle_gradient(n_water, n_pa, seed):
    p = problem(n_water, n_pa, seed)
    g, gx = oracle.problem_inputs(p)
    return oracle.gradient(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", CASES)
def test_gradient_vs_oracle(torch, case, prec):
    from paper_2208_14639_amd import vv10
    _say("gradient", prec, case)
    p = problem(*case)
    with vv10.Plan(p, prec=prec) as pl:
        g = pl.gradient(p.rho_x, p.grad_rho_x)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
    err = normwise(g, oracle_gradient(*case))
    _say("   normwise error", err)
    assert err < (TOL64 if prec == "fp64" else V_NORM)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_gradient_equals_hessian_gradient(torch, prec):
    from paper_2208_14639_amd import vv10
    p = problem(2, 37, 5)
    with vv10.Plan(p, prec=prec) as pl:
        g1 = pl.gradient(p.rho_x, p.grad_rho_x)
        g2 = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)["grad"]
        g3 = pl.gradient(p.rho_x, p.grad_rho_x)
        torch.cuda.synchronize()
        g1, g2, g3 = (x.cpu().numpy() for x in (g1, g2, g3))
    assert (g1 == g3).all()                      # deterministic, unaffected by the Hessian call
    assert normwise(g1, g2) < (1e-12 if prec == "fp64" else 2 * V_NORM)


def test_gradient_errors(torch):
    from paper_2208_14639_amd import vv10
    p = problem(1, 8, 11)
    with vv10.Plan(p, prec="fp64") as pl:
        rx = torch.as_tensor(p.rho_x, device="cuda")
        gx = torch.as_tensor(p.grad_rho_x, device="cuda")
        g = torch.empty(3 * p.n_atom, dtype=torch.float64, device="cuda")
        for n_pert, a, b, c in ((3 * p.n_atom - 1, rx, gx, g), (3 * p.n_atom, None, gx, g),
                                (3 * p.n_atom, rx, gx, None)):
            with pytest.raises(vv10.VV10Error) as ei:
                vv10.vv10_gradient(pl.handle, n_pert, a, b, c)
            assert ei.value.status == vv10.VV10_E_ARG
        vv10.vv10_gradient(pl.handle, 3 * p.n_atom, rx, gx, g)
        torch.cuda.synchronize()
        assert normwise(g.cpu().numpy(), oracle_gradient(1, 8, 11)) < TOL64
