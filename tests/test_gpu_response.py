"""vv10_trial_response -- the VV10 part of the contracted orbital Hessian for
trial densities (Section II.B, f^{rho,t} and f^{gamma,t}) -- against the
FP64 oracle, through the C ABI."""
import functools
import sys

import numpy as np
import pytest

import oracle
from gpu_util import normwise, problem
from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
RESP_NORM = {"fp32": 1e-5, "bf16x3": 5e-5}

# (n_water, n_pa, seed, n_t): tiny; ragged points and columns; the dimer
# workload; n_t = 150 is one group of ten 16-column blocks (the eight-wave
# split-BF16 form), n_t = 200 spans two column groups in every mode
CASES = [(1, 8, 11, 1), (2, 37, 5, 7), (2, 700, 1001, 18), (1, 150, 23, 150), (1, 200, 21, 200)]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@functools.lru_cache(maxsize=8)
def trial(n_water, n_pa, seed, n_t):
    p = problem(n_water, n_pa, seed)
    return inputs.trial_densities(p, n_t, seed + 100)


@functools.lru_cache(maxsize=8)
def oracle_response(n_water, n_pa, seed, n_t, i0=0, i1=None):
    p = problem(n_water, n_pa, seed)
    rt, gt = trial(n_water, n_pa, seed, n_t)
    g = oracle.gamma(p.grad_rho)
    return oracle.response_rows(i0, p.n_grid if i1 is None else i1, p.coords, p.weights, p.rho, g,
                                p.b, p.C, rt, oracle.gamma_x(p.grad_rho, gt))


def _response(torch, case, prec):
    from paper_2208_14639_amd import vv10
    p = problem(*case[:3])
    rt, gt = trial(*case)
    with vv10.Plan(p, prec=prec) as pl:
        fr, fg = pl.trial_response(rt, gt)
        torch.cuda.synchronize()
        return fr.cpu().numpy(), fg.cpu().numpy()


@pytest.mark.parametrize("case", CASES)
def test_trial_response_fp64(torch, case):
    _say("trial response fp64", case)
    fr, fg = _response(torch, case, "fp64")
    Yr, Yg = oracle_response(*case)
    assert normwise(fr, Yr) < TOL64
    assert normwise(fg, Yg) < TOL64


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", CASES)
def test_trial_response_mixed(torch, case, prec):
    _say("trial response", prec, case)
    fr, fg = _response(torch, case, prec)
    Yr, Yg = oracle_response(*case)
    errs = (normwise(fr, Yr), normwise(fg, Yg))
    _say("   errors", errs)
    assert max(errs) <= RESP_NORM[prec], errs


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_trial_response_equals_hessian_response_rows(torch, prec):
    """With the nuclear perturbations as trial densities the two entry points
    evaluate the same sums (the Hessian call's response rows)."""
    from paper_2208_14639_amd import vv10
    p = problem(2, 37, 5)
    with vv10.Plan(p, prec=prec) as pl:
        out = pl.hessian_terms(p.rho_x, p.grad_rho_x, resp=True)
        fr, fg = pl.trial_response(p.rho_x, p.grad_rho_x)
        torch.cuda.synchronize()
        tol = 1e-12 if prec == "fp64" else 2 * RESP_NORM[prec]
        assert normwise(fr.cpu().numpy(), out["resp_rho"].cpu().numpy()) < tol
        assert normwise(fg.cpu().numpy(), out["resp_gamma"].cpu().numpy()) < tol


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_trial_response_repeat_and_resize(torch, prec):
    """Repeated calls reuse the cached pair integrals and reproduce the first
    call bitwise, also after the workspace was rebuilt for another n_t and on
    a fresh plan."""
    from paper_2208_14639_amd import vv10
    case = (2, 37, 5, 7)
    p = problem(*case[:3])
    rt, gt = trial(*case)
    with vv10.Plan(p, prec=prec) as pl:
        a = [x.cpu().numpy() for x in pl.trial_response(rt, gt)]
        b = [x.cpu().numpy() for x in pl.trial_response(rt, gt)]
        c = [x.cpu().numpy() for x in pl.trial_response(rt[:3], gt[:3])]
        d = [x.cpu().numpy() for x in pl.trial_response(rt, gt)]
    with vv10.Plan(p, prec=prec) as pl:
        e = [x.cpu().numpy() for x in pl.trial_response(rt, gt)]
    for k in range(2):
        assert np.array_equal(a[k], b[k])
        assert np.array_equal(a[k], d[k])
        assert np.array_equal(a[k], e[k])
        assert c[k].shape == (3, p.n_grid)
    # the three-column call gives the same columns within rounding
    assert normwise(c[0], a[0][:3]) < (1e-12 if prec == "fp64" else 2 * RESP_NORM[prec])


def test_trial_response_errors(torch):
    from paper_2208_14639_amd import vv10
    p = problem(1, 8, 11)
    rt, gt = trial(1, 8, 11, 1)
    with vv10.Plan(p, prec="fp64") as pl:
        r = torch.as_tensor(rt, device="cuda")
        g = torch.as_tensor(gt, device="cuda")
        fr = torch.full((1, p.n_grid), 7.0, dtype=torch.float64, device="cuda")
        fg = torch.full_like(fr, 7.0)
        vv10.vv10_trial_response(pl.handle, 0, r, g, fr, fg)           # no-op
        torch.cuda.synchronize()
        assert bool((fr == 7.0).all()) and bool((fg == 7.0).all())
        for bad in (-1, 65537):
            with pytest.raises(vv10.VV10Error) as ei:
                vv10.vv10_trial_response(pl.handle, bad, r, g, fr, fg)
            assert ei.value.status == vv10.VV10_E_ARG
        with pytest.raises(vv10.VV10Error) as ei:
            vv10.vv10_trial_response(pl.handle, 1, None, g, fr, fg)
        assert ei.value.status == vv10.VV10_E_ARG
        # the plan is still usable
        vv10.vv10_trial_response(pl.handle, 1, r, g, fr, fg)
        torch.cuda.synchronize()
        Yr, _ = oracle_response(1, 8, 11, 1)
        assert normwise(fr.cpu().numpy(), Yr) < TOL64
    assert vv10.vv10_response_footprint_bytes(27000, 54, vv10.VV10_FP64) > 0
    assert vv10.vv10_response_footprint_bytes(0, 54, vv10.VV10_FP64) == 0


def test_trial_response_hexamer_sampled_rows(torch):
    """Full hexamer size (N = 27000, n_t = 54, split-BF16 as timed): sampled
    rows against the oracle, which can evaluate single rows."""
    from paper_2208_14639_amd import vv10
    case = (6, 1500, 1002, 54)
    p = problem(*case[:3])
    rt, gt = trial(*case)
    with vv10.Plan(p, prec="bf16x3") as pl:
        fr, fg = pl.trial_response(rt, gt)
        torch.cuda.synchronize()
        fr, fg = fr.cpu().numpy(), fg.cpu().numpy()
    # normwise against the largest magnitude of the whole output
    sr, sg = np.max(np.abs(fr)), np.max(np.abs(fg))
    for i0 in (0, 13511, p.n_grid - 9):
        i1 = min(p.n_grid, i0 + 9)
        _say("hexamer rows", i0, i1)
        Yr, Yg = oracle_response(*case, i0, i1)
        assert np.max(np.abs(fr[:, i0:i1] - Yr)) <= RESP_NORM["bf16x3"] * sr
        assert np.max(np.abs(fg[:, i0:i1] - Yg)) <= RESP_NORM["bf16x3"] * sg
