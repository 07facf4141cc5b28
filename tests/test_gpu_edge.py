"""Edge cases through the C ABI: an atom without grid points, grids of one to
three points, and weights that move with the nuclei on a sparse grid.  The
largest single configuration (the water 20-mer) has its own test file."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import normwise
from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _oracle_all(p):
    g, gx = oracle.problem_inputs(p)
    e0, fr0, fg0 = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
    H0, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                 p.rho_x, gx)
    G0 = oracle.gradient(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
    return e0, fr0, fg0, H0, G0


def _check(torch, p, prec="fp64"):
    from paper_2208_14639_amd import vv10
    e0, fr0, fg0, H0, G0 = _oracle_all(p)
    with vv10.Plan(p, prec=prec) as pl:
        e, fr, fg = pl.energy_potential()
        out = pl.hessian_terms(p.rho_x, p.grad_rho_x, grad=True)
        g = pl.gradient(p.rho_x, p.grad_rho_x)
        torch.cuda.synchronize()
        got = (e.item(), fr.cpu().numpy(), fg.cpu().numpy(), out["hess"].cpu().numpy(),
               out["grad"].cpu().numpy(), g.cpu().numpy())
    errs = dict(energy=abs(got[0] - e0) / abs(e0), f_rho=normwise(got[1], fr0),
                f_gamma=normwise(got[2], fg0), hess=normwise(got[3], H0),
                grad=normwise(got[4], G0), grad_only=normwise(got[5], G0))
    hess_abs = float(np.max(np.abs(got[3] - H0)))
    _say("   ", prec, errs, "hess max abs", hess_abs)
    return errs, hess_abs


def test_atom_without_points(torch):
    """A water dimer whose second oxygen carries no grid points: its segment
    is empty, its perturbations still move density at every other point."""
    rng = np.random.default_rng(41)
    mol = inputs.water_cluster(2, rng)
    ao, off, r = inputs.atom_grid(mol.n_atom, 45, rng)
    keep = ao != 3
    p = inputs.build_problem(mol, ao[keep], off[keep], r[keep])
    assert 3 not in set(p.atom_of.tolist()) and p.n_atom == 6
    errs, _ = _check(torch, p)
    assert max(errs.values()) < TOL64
    for prec in ("fp32", "bf16x3"):
        errs, hess_abs = _check(torch, p, prec)
        assert errs["energy"] < 1e-6 and hess_abs < 1e-5 and errs["grad"] < 1e-5, prec


@pytest.mark.parametrize("n_pa", [1, 2, 3])
def test_few_points(torch, n_pa):
    """One water with n_pa points per atom (N = 3 n_pa): every tile and split
    is mostly padding."""
    p = inputs.make_problem(1, n_pa, 60 + n_pa)
    errs, _ = _check(torch, p)
    assert max(errs.values()) < TOL64


def _weighted(torch, p, prec):
    from paper_2208_14639_amd import vv10
    with vv10.Plan(p, prec=prec) as pl:
        out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, grad=True, fock=True, w_x=p.w_x,
                               w_coef=True)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}


def _oracle_weighted(p):
    g, gx = oracle.problem_inputs(p)
    args = (p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
    H, _ = oracle.hessian_terms(*args, w_x=p.w_x)
    G = oracle.gradient(*args, w_x=p.w_x)
    vr, vg = oracle.fock_nuclear_terms(*args, w_x=p.w_x)
    return dict(hess=H, grad=G, fock_rho=vr, fock_gamma=vg,
                w_coef=oracle.weight_coefficients(p.coords, p.weights, p.rho, g, p.b, p.C))


def test_becke_atom_without_points(torch):
    """Becke weights on a dimer whose second oxygen has no grid points: its
    cell function still enters every other point's weight, so its
    perturbations carry weight derivatives everywhere."""
    rng = np.random.default_rng(41)
    mol = inputs.water_cluster(2, rng)
    ao, off, r = inputs.atom_grid(mol.n_atom, 45, rng)
    keep = ao != 3
    p = inputs.build_problem(mol, ao[keep], off[keep], r[keep], weights="becke")
    assert np.max(np.abs(p.w_x[9:12])) > 0
    ref = _oracle_weighted(p)
    got = _weighted(torch, p, "fp64")
    errs = {k: normwise(got[k], ref[k]) for k in ref}
    _say("    becke, atom without points", errs)
    assert max(errs.values()) < TOL64


@pytest.mark.parametrize("n_pa", [1, 3])
def test_becke_few_points(torch, n_pa):
    p = inputs.make_problem(1, n_pa, 70 + n_pa, weights="becke")
    ref = _oracle_weighted(p)
    got = _weighted(torch, p, "fp64")
    errs = {k: normwise(got[k], ref[k]) for k in ref}
    assert max(errs.values()) < TOL64, errs


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_screening_several_column_groups(torch, prec):
    """15 waters (P = 135: nine 16-column blocks, two column groups in FP64,
    one in split-BF16), 40 points per atom in shell order: screened response
    rows stay within the unscreened ones' bound of the oracle."""
    from paper_2208_14639_amd import vv10
    p = inputs.make_problem(15, 40, 91, radial_order=True)
    g, gx = oracle.problem_inputs(p)
    Yr0, Yg0 = oracle.response_rows(0, p.n_grid, p.coords, p.weights, p.rho, g, p.b, p.C,
                                    p.rho_x, gx)
    res = {}
    for tau in (0.0, 1e-8):
        with vv10.Plan(p, prec=prec, screening=tau) as pl:
            out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, resp=True)
            tiles = vv10.vv10_get_tiles(pl.handle)
            stats = vv10.vv10_screening_stats(pl.handle) if tau else None
            torch.cuda.synchronize()
            res[tau] = {k: v.cpu().numpy() for k, v in out.items()}
        _say("   ", prec, "tau", tau, "tiles", tiles, "stats", stats)
    bound = TOL64 if prec == "fp64" else 5e-5
    assert normwise(res[0.0]["resp_rho"], Yr0) < bound
    assert normwise(res[1e-8]["resp_rho"], res[0.0]["resp_rho"]) < 3e-6
    assert normwise(res[1e-8]["resp_gamma"], res[0.0]["resp_gamma"]) < 3e-6
    assert normwise(res[1e-8]["hess"], res[0.0]["hess"]) < 3e-6
