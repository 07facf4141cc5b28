"""The largest request of the served stream through the C ABI: 30 waters at
2500 points per atom (N = 225000, P = 270; two column groups of nine
16-column blocks in the mixed modes, three of six in FP64).  The
Hessian terms (Section II.B) in split-BF16 as served and in FP64 are checked
on the response rows of the grid's ragged tail, which the oracle evaluates
one at a time, on properties that hold at any size (exact symmetry, every
row summing to zero over the atoms), and against each other."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import normwise
from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
E_REL, H_ABS, RESP_NORM = 1e-6, 1e-5, 5e-5


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def test_largest_request(torch):
    from paper_2208_14639_amd import vv10
    _say("   generating N = 225000, P = 270")
    p = inputs.make_problem(30, 2500, 4242)
    n, P = p.n_grid, p.n_pert
    res = {}
    for prec in ("bf16x3", "fp64"):
        _say("   running", prec)
        with vv10.Plan(p, prec=prec, tiles="auto" if prec == "bf16x3" else None) as pl:
            out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, resp=True, energy=True)
            tiles = vv10.vv10_get_tiles(pl.handle)
            torch.cuda.synchronize()
            res[prec] = dict(hess=out["hess"].cpu().numpy(), energy=out["energy"].item(),
                             rr=out["resp_rho"][:, n - 4:].cpu().numpy(),
                             rg=out["resp_gamma"][:, n - 4:].cpu().numpy(),
                             rr_max=float(out["resp_rho"].abs().max()),
                             rg_max=float(out["resp_gamma"].abs().max()))
            del out
        _say("   ", prec, "tiles", tiles)
    for prec, r in res.items():
        H = r["hess"]
        assert np.array_equal(H, H.T), prec
        rows = H.reshape(P, p.n_atom, 3).sum(axis=1)
        _say("   ", prec, "translational residual", np.max(np.abs(rows)), "of", np.max(np.abs(H)))
        assert np.max(np.abs(rows)) <= (1e-10 if prec == "fp64" else 1e-5) * np.max(np.abs(H))
    b, f = res["bf16x3"], res["fp64"]
    dh = float(np.max(np.abs(b["hess"] - f["hess"])))
    de = abs(b["energy"] - f["energy"]) / abs(f["energy"])
    _say("    split-BF16 vs FP64: hess max abs", dh, "energy rel", de)
    assert dh <= H_ABS and de <= E_REL
    _say("   oracle rows", n - 4, "..", n)
    g, gx = oracle.problem_inputs(p)
    Yr, Yg = oracle.response_rows(n - 4, n, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
    e64 = (np.max(np.abs(f["rr"] - Yr)) / np.max(np.abs(Yr)),
           np.max(np.abs(f["rg"] - Yg)) / np.max(np.abs(Yg)))
    eb = (np.max(np.abs(b["rr"] - Yr)) / b["rr_max"], np.max(np.abs(b["rg"] - Yg)) / b["rg_max"])
    _say("    rows vs oracle: fp64", e64, "split-BF16 (of the largest row entry)", eb)
    assert max(e64) < TOL64
    assert max(eb) <= RESP_NORM
