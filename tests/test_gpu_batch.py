"""Batched evaluation (one HIP graph with a persistent contraction) against
the single-molecule path and the oracle."""
import sys

import numpy as np
import pytest

from gpu_util import normwise, relerr
import oracle
from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_problems(n_mol, seed, n_pa=(150, 400), waters=(1, 4)):
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n_mol):
        k = int(rng.integers(waters[0], waters[1] + 1))
        pa = int(rng.integers(n_pa[0], n_pa[1] + 1))
        out.append(inputs.make_problem(k, pa, seed * 100 + m))
    return out


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_batch_equals_single_molecule_path(torch, prec):
    from paper_2208_14639_amd import vv10
    probs = batch_problems(5, 77)
    with vv10.Batch(probs, prec=prec) as b:
        e, blocks = b.run()
        torch.cuda.synchronize()
        n_items, n_wg = b.info()
        _say(prec, "items", n_items, "workgroups", n_wg)
        e = e.cpu().numpy()
        Hb = [h.cpu().numpy() for h in blocks]
    bitwise = True
    for m, p in enumerate(probs):
        with vv10.Plan(p, prec=prec) as pl:
            out = pl.hessian_terms(p.rho_x, p.grad_rho_x)
            es, _, _ = pl.energy_potential()
            torch.cuda.synchronize()
            H = out["hess"].cpu().numpy()
        bitwise &= bool(np.array_equal(H, Hb[m]))
        assert normwise(Hb[m], H) < 1e-13, (m, normwise(Hb[m], H))
        # the batch's energy comes from the Hessian-mode pair pass, the single
        # path's from the energy pass: same sums, different split boundaries
        assert relerr(e[m], es.item()) < (1e-13 if prec == "fp64" else 1e-7)
    # same tile functions, same per-item output slabs, same reduction order
    assert bitwise


def test_batch_fp64_matches_oracle(torch):
    from paper_2208_14639_amd import vv10
    probs = batch_problems(4, 78, n_pa=(60, 120))
    with vv10.Batch(probs, prec="fp64") as b:
        e, blocks = b.run()
        torch.cuda.synchronize()
        e = e.cpu().numpy()
        Hb = [h.cpu().numpy() for h in blocks]
    for m, p in enumerate(probs):
        g, gx = oracle.problem_inputs(p)
        H0, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b,
                                     p.C, p.rho_x, gx)
        e0, _, _ = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        assert normwise(Hb[m], H0) < 1e-10
        assert relerr(e[m], e0) < 1e-10


def test_batch_mixed_bounds_vs_oracle(torch):
    from paper_2208_14639_amd import vv10
    probs = batch_problems(4, 79, n_pa=(60, 120))
    with vv10.Batch(probs, prec="bf16x3") as b:
        e, blocks = b.run()
        torch.cuda.synchronize()
        e = e.cpu().numpy()
        Hb = [h.cpu().numpy() for h in blocks]
    for m, p in enumerate(probs):
        g, gx = oracle.problem_inputs(p)
        H0, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b,
                                     p.C, p.rho_x, gx)
        e0, _, _ = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        assert np.max(np.abs(Hb[m] - H0)) <= 1e-5
        assert relerr(e[m], e0) <= 1e-6


@pytest.mark.parametrize("prec,tiles", [("bf16x3", None), ("bf16x3", [(3, 0), (1, 0), (1, 0), (2, 0)]),
                                        ("fp32", None), ("fp64", None)])
def test_batch_wide_items(torch, prec, tiles):
    """Molecules of eight or more column blocks (14, 17 and 21 waters: 8, 10
    and 12 blocks) beside a 2-water one.  Split-BF16 runs the wide ones'
    contraction items in the eight-wave persistent kernel and the small
    one's in the four-wave kernel; FP32 runs all of them in its four-wave
    kernel at up to twelve blocks, FP64 in two column groups above eight.
    Every Hessian equals the single path's bitwise (the same tile functions),
    and the largest is within the bounds of the oracle (Section II.B E^{AB})."""
    from paper_2208_14639_amd import vv10
    probs = [inputs.make_problem(14, 40, 901), inputs.make_problem(2, 150, 902),
             inputs.make_problem(21, 30, 903), inputs.make_problem(17, 30, 904)]
    with vv10.Batch(probs, prec=prec, tiles=tiles) as b:
        e, blocks = b.run()
        torch.cuda.synchronize()
        n_items, n_wg = b.info()
        _say("wide batch: items", n_items, "workgroups", n_wg)
        Hb = [h.cpu().numpy() for h in blocks]
    for m, p in enumerate(probs):
        with vv10.Plan(p, prec=prec, tiles=None if tiles is None else tiles[m]) as pl:
            H = pl.hessian_terms(p.rho_x, p.grad_rho_x)["hess"].cpu().numpy()
            torch.cuda.synchronize()
        assert np.array_equal(H, Hb[m]), (m, normwise(Hb[m], H))
    p = probs[2]
    g, gx = oracle.problem_inputs(p)
    H0, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                 p.rho_x, gx)
    if prec == "fp64":
        assert normwise(Hb[2], H0) < 1e-10
    else:
        assert np.max(np.abs(Hb[2] - H0)) <= 1e-5


def test_graph_replays_with_eager_work_between(torch):
    """Each replay of the captured graph equals the first result, with eager
    work (another plan's evaluation and host syncs) between the replays."""
    from paper_2208_14639_amd import vv10
    probs = batch_problems(3, 80)
    other = inputs.make_problem(2, 100, 5)
    with vv10.Batch(probs, prec="bf16x3") as b:
        e0, blocks0 = b.run()
        torch.cuda.synchronize()
        ref_e = e0.clone()
        ref_h = b.hess.clone()
        for rep in range(4):
            with vv10.Plan(other, prec="fp64") as pl:
                pl.hessian_terms(other.rho_x, other.grad_rho_x)
            b.energy.fill_(0.0)
            b.hess.fill_(0.0)
            torch.cuda.synchronize()
            b.run()
            torch.cuda.synchronize()
            assert torch.equal(b.energy, ref_e), rep
            assert torch.equal(b.hess, ref_h), rep


def test_tiles_override_consistent(torch):
    from paper_2208_14639_amd import vv10
    p = inputs.make_problem(3, 400, 81)
    with vv10.Plan(p, prec="bf16x3") as pl:
        Ha = pl.hessian_terms(p.rho_x, p.grad_rho_x)["hess"].cpu().numpy()
    with vv10.Plan(p, prec="bf16x3", tiles=(5, 2)) as pl:
        Hb = pl.hessian_terms(p.rho_x, p.grad_rho_x)["hess"].cpu().numpy()
    assert np.max(np.abs(Ha - Hb)) < 1e-6
