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


# ---------------------------------------------------------------------------
# Mixed precision: FP32 pair arithmetic, FP32 or split-BF16 MFMA contraction,
# FP64 accumulation across tiles.  Bounds: energy <= 1e-6 relative, every
# Hessian element <= 1e-5 au absolute; potential and gradient <= 1e-5
# normwise; response rows <= 1e-5 (FP32) and 5e-5 (split-BF16, whose
# operands carry about 2^-16 relative error each and whose small rows do not
# average it out) normwise.
# ---------------------------------------------------------------------------
MIXED = ["fp32", "bf16x3"]
E_REL, H_ABS, V_NORM = 1e-6, 1e-5, 1e-5
RESP_NORM = {"fp32": 1e-5, "bf16x3": 5e-5}


@pytest.mark.parametrize("prec", MIXED)
@pytest.mark.parametrize("case", CASES)
def test_mixed_precision_bounds(torch, case, prec):
    _say("mixed", prec, case)
    p = problem(*case)
    with _plan(torch, case, prec) as pl:
        e, fr, fg = pl.energy_potential()
        out = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True, resp=True)
        torch.cuda.synchronize()
    e0, fr0, fg0 = oracle_energy(*case)
    H0, G0, (Yr0, Yg0) = oracle_hessian(*case)
    H = out["hess"].cpu().numpy()
    errs = dict(
        energy_rel=relerr(e.item(), e0),
        f_rho=normwise(fr.cpu().numpy(), fr0),
        f_gamma=normwise(fg.cpu().numpy(), fg0),
        grad=normwise(out["grad"].cpu().numpy(), G0),
        resp_rho=normwise(out["resp_rho"].cpu().numpy(), Yr0),
        resp_gamma=normwise(out["resp_gamma"].cpu().numpy(), Yg0),
        hess_max_abs=float(np.max(np.abs(H - H0))),
        hess_normwise=normwise(H, H0),
    )
    _say("  errors", errs)
    assert errs["energy_rel"] <= E_REL
    assert errs["hess_max_abs"] <= H_ABS
    for k in ("f_rho", "f_gamma", "grad"):
        assert errs[k] <= V_NORM, (k, errs[k])
    for k in ("resp_rho", "resp_gamma"):
        assert errs[k] <= RESP_NORM[prec], (k, errs[k])
    assert np.array_equal(H, H.T)


@pytest.mark.parametrize("prec", MIXED)
def test_mixed_deterministic(torch, prec):
    case = CASES[2]
    p = problem(*case)
    with _plan(torch, case, prec) as pl:
        a = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)
        b = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)
        torch.cuda.synchronize()
        assert torch.equal(a["hess"], b["hess"]) and torch.equal(a["grad"], b["grad"])
