"""Error handling of the C ABI on the GPU: bad inputs are rejected with the
documented status before any output is written."""
import numpy as np
import pytest

from gpu_util import problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vv():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_14639_amd import vv10
    return vv10


def _dev(a):
    import torch
    return torch.as_tensor(a).cuda().contiguous()


def _prepare(vv, p, **over):
    import torch
    args = dict(coords=p.coords, weights=p.weights, atom_of=p.atom_of.astype(np.int32),
                rho=p.rho, grad_rho=p.grad_rho)
    args.update(over)
    t = {k: _dev(v) for k, v in args.items()}
    n_atom = over.get("n_atom", p.n_atom)
    return vv.vv10_prepare(p.b, p.C, p.n_grid, n_atom, t["coords"], t["weights"], t["atom_of"],
                           t["rho"], t["grad_rho"], vv.VV10_FP64)


def test_bad_density(vv):
    p = problem(1, 8, 11)
    rho = p.rho.copy()
    rho[5] = -1.0
    with pytest.raises(vv.VV10Error) as e:
        _prepare(vv, p, rho=rho)
    assert e.value.status == vv.VV10_E_DENSITY
    rho[5] = np.nan
    with pytest.raises(vv.VV10Error) as e:
        _prepare(vv, p, rho=rho)
    assert e.value.status == vv.VV10_E_DENSITY


def test_unsorted_grid(vv):
    p = problem(1, 8, 11)
    ao = p.atom_of.copy()
    ao[0], ao[-1] = ao[-1], ao[0]
    with pytest.raises(vv.VV10Error) as e:
        _prepare(vv, p, atom_of=ao)
    assert e.value.status == vv.VV10_E_GRID_ORDER


def test_atom_index_out_of_range(vv):
    p = problem(1, 8, 11)
    ao = p.atom_of.copy()
    ao[-1] = 7
    with pytest.raises(vv.VV10Error) as e:
        _prepare(vv, p, atom_of=ao)
    assert e.value.status == vv.VV10_E_ARG


def test_wrong_n_pert_and_null_outputs(vv):
    import torch
    p = problem(1, 8, 11)
    h = _prepare(vv, p)
    try:
        rx, gx = _dev(p.rho_x), _dev(p.grad_rho_x)
        H = torch.full((9, 9), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(vv.VV10Error) as e:
            vv.vv10_hessian_terms(h, 6, rx, gx, H)
        assert e.value.status == vv.VV10_E_ARG
        with pytest.raises(vv.VV10Error) as e:
            vv.vv10_hessian_terms(h, 9, rx, gx, None)
        assert e.value.status == vv.VV10_E_ARG
        with pytest.raises(vv.VV10Error) as e:
            vv.vv10_energy_potential(h, None)
        assert e.value.status == vv.VV10_E_ARG
        torch.cuda.synchronize()
        assert torch.all(H == 7.0)      # nothing written on error
    finally:
        vv.vv10_destroy(h)


def test_single_atom(vv):
    """One atom carrying its own grid: every nuclear displacement moves the
    whole system rigidly, so rho^x = 0, there are no grid-position pairs,
    and the Hessian terms vanish identically."""
    import torch
    from paper_2208_14639_amd import inputs
    rng = np.random.default_rng(3)
    mol = inputs.Molecule(Z=np.array([8]), zeta=np.array([2.0]), R=np.zeros((1, 3)))
    ao, off, r = inputs.atom_grid(1, 300, rng)
    p = inputs.build_problem(mol, ao, off, r)
    with vv.Plan(p) as pl:
        out = pl.hessian_terms(p.rho_x, p.grad_rho_x)
        torch.cuda.synchronize()
        H = out["hess"].cpu().numpy()
    assert np.all(H == 0.0)
