"""vv10_energy_potential_noalloc (the entry point that allocates nothing:
its working memory is the library's static scratch array) against the plan
path vv10_prepare + vv10_energy_potential, through the C ABI: bitwise equal
energy and potential, on two calls in a row, the second with a smaller grid
(the scratch array keeps the first call's contents), in every precision;
invalid densities reported through the status word with no output written;
grids beyond the scratch array rejected."""
import numpy as np
import pytest

from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _dev(torch, p):
    f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).cuda().contiguous()
    return dict(coords=f64(p.coords), w=f64(p.weights), rho=f64(p.rho), grad=f64(p.grad_rho),
                atom_of=torch.as_tensor(p.atom_of, dtype=torch.int32).cuda().contiguous())


def _plan_path(torch, vv10, p, d, prec):
    stream = torch.cuda.current_stream().cuda_stream
    h = vv10.vv10_prepare(p.b, p.C, p.n_grid, p.n_atom, d["coords"], d["w"], d["atom_of"],
                          d["rho"], d["grad"], prec, stream)
    try:
        e = torch.empty(1, dtype=torch.float64, device="cuda")
        fr = torch.empty(p.n_grid, dtype=torch.float64, device="cuda")
        fg = torch.empty_like(fr)
        vv10.vv10_energy_potential(h, e, fr, fg)
        torch.cuda.synchronize()
    finally:
        vv10.vv10_destroy(h)
    return e.cpu().numpy(), fr.cpu().numpy(), fg.cpu().numpy()


def _noalloc(torch, vv10, p, d, prec, rho=None):
    stream = torch.cuda.current_stream().cuda_stream
    e = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    fr = torch.full((p.n_grid,), float("nan"), dtype=torch.float64, device="cuda")
    fg = torch.full_like(fr, float("nan"))
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    vv10.vv10_energy_potential_noalloc(p.b, p.C, p.n_grid, p.n_atom, d["coords"], d["w"],
                                       d["atom_of"], d["rho"] if rho is None else rho, d["grad"],
                                       prec, stream, e, fr, fg, status)
    torch.cuda.synchronize()
    return e.cpu().numpy(), fr.cpu().numpy(), fg.cpu().numpy(), int(status.item())


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_equals_plan_path_twice(torch, prec):
    from paper_2208_14639_amd import vv10
    pr = vv10.PRECISIONS[prec]
    big = inputs.make_problem(2, 700, 1001)      # N = 4200
    small = inputs.make_problem(1, 300, 77)      # N = 900, after the larger call
    for p in (big, small):
        d = _dev(torch, p)
        ref = _plan_path(torch, vv10, p, d, pr)
        got = _noalloc(torch, vv10, p, d, pr)
        assert got[3] == vv10.VV10_OK
        for a, b in zip(got[:3], ref):
            assert np.array_equal(a, b), (prec, p.n_grid)


def test_noalloc_invalid_density_writes_nothing(torch):
    from paper_2208_14639_amd import vv10
    p = inputs.make_problem(1, 200, 78)
    d = _dev(torch, p)
    bad = d["rho"].clone()
    bad[17] = -1.0
    e, fr, fg, status = _noalloc(torch, vv10, p, d, vv10.VV10_FP64, rho=bad)
    assert status == vv10.VV10_E_DENSITY
    assert np.isnan(e).all() and np.isnan(fr).all() and np.isnan(fg).all()
    # a valid call right after it is unaffected
    e, fr, fg, status = _noalloc(torch, vv10, p, d, vv10.VV10_FP64)
    ref = _plan_path(torch, vv10, p, d, vv10.VV10_FP64)
    assert status == vv10.VV10_OK and np.array_equal(e, ref[0]) and np.array_equal(fr, ref[1])


def test_noalloc_rejects_grids_beyond_scratch(torch):
    from paper_2208_14639_amd import vv10
    limit = vv10.VV10_NOALLOC_SCRATCH_BYTES
    assert vv10.vv10_noalloc_bytes(250000, 90) <= limit < vv10.vv10_noalloc_bytes(260000, 90)
    p = inputs.make_problem(1, 10, 79)
    d = _dev(torch, p)
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(vv10.VV10Error) as ex:
        # the size check comes before any launch, so the small arrays are never read
        vv10.vv10_energy_potential_noalloc(p.b, p.C, 260000, 90, d["coords"], d["w"], d["atom_of"],
                                           d["rho"], d["grad"], vv10.VV10_FP64,
                                           torch.cuda.current_stream().cuda_stream, e)
    assert ex.value.status == vv10.VV10_E_ARG
