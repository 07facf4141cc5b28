"""vv10_nuclear_terms: the grid-level coefficients of the Fock nuclear
derivative (Section II.B, F^A_G + F^A_gr) against the FP64 oracle, and the
output subsets against vv10_hessian_terms."""
import functools
import sys

import numpy as np
import pytest

import oracle
from gpu_util import normwise, problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
FOCK_NORM = {"fp32": 1e-5, "bf16x3": 5e-5}
CASES = [(1, 8, 11), (2, 37, 5), (2, 700, 1001)]
# wide column groups: eight (14 waters, the eight-wave split-BF16 form) and
# twelve 16-column blocks (21 waters), 30-40 points per atom
WIDE = [(14, 40, 614), (21, 30, 621)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@functools.lru_cache(maxsize=8)
def oracle_fock(n_water, n_pa, seed):
    p = problem(n_water, n_pa, seed)
    g, gx = oracle.problem_inputs(p)
    return oracle.fock_nuclear_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                     p.rho_x, gx)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", CASES + WIDE)
def test_fock_terms_vs_oracle(torch, case, prec):
    from paper_2208_14639_amd import vv10
    _say("fock terms", prec, case)
    p = problem(*case)
    with vv10.Plan(p, prec=prec) as pl:
        out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=False, fock=True)
        torch.cuda.synchronize()
        vr, vg = out["fock_rho"].cpu().numpy(), out["fock_gamma"].cpu().numpy()
    vr0, vg0 = oracle_fock(*case)
    errs = (normwise(vr, vr0), normwise(vg, vg0))
    _say("   normwise errors", errs)
    assert max(errs) < (TOL64 if prec == "fp64" else FOCK_NORM[prec])


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_output_subsets_agree(torch, prec):
    """Every subset of outputs gives the same values, bitwise, as
    vv10_hessian_terms (same launches, outputs only switched on or off); no
    output at all is a no-op."""
    from paper_2208_14639_amd import vv10
    p = problem(2, 37, 5)
    with vv10.Plan(p, prec=prec) as pl:
        ref = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True, resp=True)
        full = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, grad=True, resp=True, fock=True)
        only_h = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True)
        only_g = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=False, grad=True)
        only_f = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=False, fock=True)
        none = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=False)
        torch.cuda.synchronize()
        c = lambda d, k: d[k].cpu().numpy()
        for k in ("hess", "grad", "resp_rho", "resp_gamma"):
            assert np.array_equal(c(full, k), c(ref, k)), k
        assert np.array_equal(c(only_h, "hess"), c(ref, "hess"))
        assert np.array_equal(c(only_g, "grad"), c(ref, "grad"))
        assert np.array_equal(c(only_f, "fock_rho"), c(full, "fock_rho"))
        assert np.array_equal(c(only_f, "fock_gamma"), c(full, "fock_gamma"))
        assert none == {}


def test_nuclear_terms_errors(torch):
    from paper_2208_14639_amd import vv10
    p = problem(1, 8, 11)
    with vv10.Plan(p, prec="fp64") as pl:
        rx = torch.as_tensor(p.rho_x, device="cuda")
        gx = torch.as_tensor(p.grad_rho_x, device="cuda")
        for n_pert, a in ((3 * p.n_atom + 1, rx), (3 * p.n_atom, None)):
            with pytest.raises(vv10.VV10Error) as ei:
                vv10.vv10_nuclear_terms(pl.handle, n_pert, a, gx,
                                        hess=torch.empty((9, 9), dtype=torch.float64, device="cuda"))
            assert ei.value.status == vv10.VV10_E_ARG
        with pytest.raises(vv10.VV10Error) as ei:
            vv10.vv10_hessian_terms(pl.handle, 3 * p.n_atom, rx, gx, None)
        assert ei.value.status == vv10.VV10_E_ARG


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", CASES)
def test_energy_potential_from_nuclear_terms(torch, case, prec):
    """One vv10_nuclear_terms call returns the energy and potential from the
    integrals its grid pass forms: against the oracle to the stated bounds,
    and against vv10_energy_potential on a fresh plan (same sums, different
    partial boundaries)."""
    from paper_2208_14639_amd import vv10
    from gpu_util import oracle_energy, oracle_hessian, relerr
    p = problem(*case)
    with vv10.Plan(p, prec=prec) as pl:
        out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, grad=True, energy=True,
                               potential=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    with vv10.Plan(p, prec=prec) as pl:
        e2, fr2, fg2 = (x.cpu().numpy() for x in pl.energy_potential())
    e0, fr0, fg0 = oracle_energy(*case)
    H0, G0, _ = oracle_hessian(*case)
    errs = dict(energy=relerr(got["energy"][0], e0), f_rho=normwise(got["f_rho"], fr0),
                f_gamma=normwise(got["f_gamma"], fg0), hess=normwise(got["hess"], H0),
                grad=normwise(got["grad"], G0), vs_energy_call=relerr(got["energy"][0], e2[0]))
    _say("   ", prec, case, errs)
    if prec == "fp64":
        assert max(v for k, v in errs.items() if k != "vs_energy_call") < TOL64
        assert errs["vs_energy_call"] < 1e-13
    else:
        assert errs["energy"] <= 1e-6 and errs["f_rho"] <= 1e-5 and errs["f_gamma"] <= 1e-5
        assert errs["vs_energy_call"] < 1e-6
        assert np.max(np.abs(got["hess"] - H0)) <= 1e-5


def test_fused_step_hexamer_as_timed(torch):
    """The benchmark's step on the hexamer workload (N = 27000, P = 54):
    split-BF16, tuned tiles, one vv10_nuclear_terms call with energy,
    potential, Hessian and gradient, against the whole oracle."""
    from paper_2208_14639_amd import vv10
    from gpu_util import oracle_energy, oracle_hessian, relerr
    case = (6, 1500, 1002)
    p = problem(*case)
    with vv10.Plan(p, prec="bf16x3", tiles="auto") as pl:
        out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, grad=True, energy=True,
                               potential=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    e0, fr0, fg0 = oracle_energy(*case)
    H0, G0, _ = oracle_hessian(*case)
    errs = dict(energy=relerr(got["energy"][0], e0), f_rho=normwise(got["f_rho"], fr0),
                f_gamma=normwise(got["f_gamma"], fg0), grad=normwise(got["grad"], G0),
                hess_abs=float(np.max(np.abs(got["hess"] - H0))))
    _say("    hexamer fused step", errs)
    assert errs["energy"] <= 1e-6 and errs["hess_abs"] <= 1e-5
    assert max(errs["f_rho"], errs["f_gamma"], errs["grad"]) <= 1e-5
    assert np.array_equal(got["hess"], got["hess"].T)
