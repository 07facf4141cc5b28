"""Streams and stage timing through the C ABI: a plan rebound to another
stream (vv10_set_stream), two plans running at once on two streams, and
per-stage timing (vv10_set_timing, vv10_set_timing_stages,
vv10_stage_times), all giving bitwise the results of a plan on the default
stream."""
import numpy as np
import pytest

from paper_2208_14639_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def prob():
    return inputs.make_problem(3, 200, 71)


def _terms(pl, p):
    out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, grad=True, energy=True,
                           potential=True)
    return out


def _host(torch, out):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_set_stream(torch, prob, prec):
    from paper_2208_14639_amd import vv10
    p = prob
    with vv10.Plan(p, prec=prec) as pl:
        ref = _host(torch, _terms(pl, p))
    s = torch.cuda.Stream()              # default priority
    with vv10.Plan(p, prec=prec) as pl:
        torch.cuda.synchronize()         # the plan's preparation is done before the rebind
        vv10.vv10_set_stream(pl.handle, s.cuda_stream)
        with torch.cuda.stream(s):
            out = _terms(pl, p)
        s.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


def test_two_plans_two_streams(torch, prob):
    """Distinct plans on distinct streams run at once; each result is
    bitwise the one of the same plan run alone."""
    from paper_2208_14639_amd import vv10
    p = prob
    q = inputs.make_problem(2, 300, 72)
    with vv10.Plan(p, prec="bf16x3") as a, vv10.Plan(q, prec="fp64") as b:
        ra, rb = _host(torch, _terms(a, p)), _host(torch, _terms(b, q))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        a = vv10.Plan(p, prec="bf16x3", stream=s1.cuda_stream)
    with torch.cuda.stream(s2):
        b = vv10.Plan(q, prec="fp64", stream=s2.cuda_stream)
    try:
        for rep in range(3):
            with torch.cuda.stream(s1):
                oa = _terms(a, p)
            with torch.cuda.stream(s2):
                ob = _terms(b, q)
            s1.synchronize()
            s2.synchronize()
            ga = {k: v.cpu().numpy() for k, v in oa.items()}
            gb = {k: v.cpu().numpy() for k, v in ob.items()}
            for k in ra:
                assert np.array_equal(ga[k], ra[k]), (rep, k)
                assert np.array_equal(gb[k], rb[k]), (rep, k)
    finally:
        a.close()
        b.close()


def test_stage_times(torch, prob):
    from paper_2208_14639_amd import vv10
    p = prob
    with vv10.Plan(p, prec="bf16x3") as pl:
        ref = _host(torch, _terms(pl, p))
        with pytest.raises(vv10.VV10Error) as ei:
            vv10.vv10_stage_times(pl.handle)
        assert ei.value.status == vv10.VV10_E_STATE
    with vv10.Plan(p, prec="bf16x3") as pl:
        vv10.vv10_set_timing(pl.handle, True)
        got = _host(torch, _terms(pl, p))
        st = vv10.vv10_stage_times(pl.handle)
        assert set(st) == set(vv10.STAGES)
        assert all(v >= 0.0 for v in st.values())
        # one fused call: the grid pass forms the pair integrals, so no pair stage
        for k in ("pert_prep", "contract", "grid", "assemble", "potential"):
            assert st[k] > 0.0, (k, st)
        assert st["pair"] == 0.0 and st["weights"] == 0.0, st
        e, fr, fg = pl.energy_potential()      # integrals kept: still no pair pass
        torch.cuda.synchronize()
        assert vv10.vv10_stage_times(pl.handle)["pair"] == 0.0
        vv10.vv10_set_timing(pl.handle, False)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    with vv10.Plan(p, prec="bf16x3") as pl:
        vv10.vv10_set_timing(pl.handle, True)
        pl.energy_potential()
        torch.cuda.synchronize()
        st = vv10.vv10_stage_times(pl.handle)
        assert st["pair"] > 0.0 and st["contract"] == 0.0, st


def test_timing_chosen_stages(torch, prob):
    """vv10_set_timing_stages brackets only the chosen stages; results stay
    bitwise the same; a mask beyond the stages is rejected."""
    from paper_2208_14639_amd import vv10
    p = prob
    with vv10.Plan(p, prec="bf16x3") as pl:
        ref = _host(torch, _terms(pl, p))
    with vv10.Plan(p, prec="bf16x3") as pl:
        with pytest.raises(vv10.VV10Error) as ei:
            vv10.vv10_set_timing_stages(pl.handle, 1 << len(vv10.STAGES))
        assert ei.value.status == vv10.VV10_E_ARG
        vv10.vv10_set_timing_stages(pl.handle, ["contract"])
        got = _host(torch, _terms(pl, p))
        st = vv10.vv10_stage_times(pl.handle)
        assert st["contract"] > 0.0, st
        assert all(v == 0.0 for k, v in st.items() if k != "contract"), st
        vv10.vv10_set_timing_stages(pl.handle, ["grid", "assemble"])
        _host(torch, _terms(pl, p))
        st2 = vv10.vv10_stage_times(pl.handle)
        assert st2["grid"] > 0.0 and st2["assemble"] > 0.0, st2
        assert st2["contract"] == st["contract"], (st, st2)   # most recent timed run
        vv10.vv10_set_timing_stages(pl.handle, 0)
        _host(torch, _terms(pl, p))
        assert vv10.vv10_stage_times(pl.handle) == st2
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
