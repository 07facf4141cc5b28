"""Parity of the HIP library (called through the C ABI) with the FP64 oracle.

FP64 path: every output within 1e-10 relative of the oracle, normwise
(max |diff| / max |oracle|) for vectors and matrices, plain relative for
the energy.
"""
import sys

import numpy as np
import pytest

from gpu_util import normwise, relerr, problem, oracle_energy, oracle_hessian

pytestmark = pytest.mark.gpu

TOL64 = 1e-10

# (n_water, n_pa, seed): tiny, ragged (N not a multiple of any tile), dimer workload, hexamer workload
CASES = [(1, 8, 11), (2, 37, 5), (2, 700, 1001), (6, 1500, 1002)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _plan(torch, case, prec="fp64"):
    from paper_2208_14639_amd import vv10
    return vv10.Plan(problem(*case), prec=prec)


@pytest.mark.parametrize("case", CASES)
def test_energy_potential_fp64(torch, case):
    _say("energy/potential fp64", case)
    with _plan(torch, case) as pl:
        e, fr, fg = pl.energy_potential()
        torch.cuda.synchronize()
        e0, fr0, fg0 = oracle_energy(*case)
        assert relerr(e.item(), e0) < TOL64
        assert normwise(fr.cpu().numpy(), fr0) < TOL64
        assert normwise(fg.cpu().numpy(), fg0) < TOL64


@pytest.mark.parametrize("case", CASES)
def test_hessian_terms_fp64(torch, case):
    _say("hessian fp64", case)
    p = problem(*case)
    with _plan(torch, case) as pl:
        out = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True, resp=True)
        torch.cuda.synchronize()
        H0, G0, (Yr0, Yg0) = oracle_hessian(*case)
        errs = dict(
            resp_rho=normwise(out["resp_rho"].cpu().numpy(), Yr0),
            resp_gamma=normwise(out["resp_gamma"].cpu().numpy(), Yg0),
            grad=normwise(out["grad"].cpu().numpy(), G0),
            hess=normwise(out["hess"].cpu().numpy(), H0),
        )
        _say("  errors", errs)
        for k, v in errs.items():
            assert v < TOL64, (k, v)
        H = out["hess"].cpu().numpy()
        assert np.array_equal(H, H.T)


def test_fp64_deterministic(torch):
    case = CASES[2]
    p = problem(*case)
    with _plan(torch, case) as pl:
        a = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)
        b = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)
        e1 = pl.energy_potential()
        e2 = pl.energy_potential()
        torch.cuda.synchronize()
        assert torch.equal(a["hess"], b["hess"]) and torch.equal(a["grad"], b["grad"])
        assert all(torch.equal(x, y) for x, y in zip(e1, e2))


def test_translational_invariance_fp64(torch):
    case = CASES[3]
    p = problem(*case)
    with _plan(torch, case) as pl:
        out = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)
        torch.cuda.synchronize()
        H = out["hess"].cpu().numpy()
        s = H.reshape(p.n_pert, p.n_atom, 3).sum(axis=1)
        assert np.max(np.abs(s)) < 1e-10 * np.max(np.abs(H))
        g = out["grad"].cpu().numpy().reshape(-1, 3).sum(axis=0)
        assert np.max(np.abs(g)) < 1e-10 * np.max(np.abs(out["grad"].cpu().numpy()))
