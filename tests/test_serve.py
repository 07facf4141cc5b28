"""Scheduling logic of the continuous-batching server, on the CPU with a
fake executor (oracle results, delays proportional to N^2 P)."""
import numpy as np
import pytest

from paper_2208_14639_amd import inputs
from fake_executor import FakeExecutor
from paper_2208_14639_amd.serve import Request, Server, percentile


def mols(n, seed=3):
    rng = np.random.default_rng(seed)
    return [inputs.make_problem(int(rng.integers(1, 3)), int(rng.integers(6, 20)), seed * 10 + k)
            for k in range(n)]


def test_percentile():
    assert percentile([1, 2, 3, 4, 5], 50) == 3
    assert percentile([1.0], 99) == 1.0
    assert abs(percentile(list(range(101)), 99) - 99.0) < 1e-12
    assert percentile([], 50) is None


def test_results_match_requests_and_budget_respected():
    ps = mols(8)
    ex = FakeExecutor(seconds_per_pair_pert=2e-8)
    budget = 3 * max(ex.footprint(p) for p in ps)
    srv = Server(ex, budget, n_slots=3)
    futs = [srv.submit(Request(k, f"m{k}", p), at=0.002 * k) for k, p in enumerate(ps)]
    peak = 0
    while srv.step():
        peak = max(peak, srv.used)
        assert srv.used <= budget
    assert peak <= budget
    import oracle
    for k, (p, f) in enumerate(zip(ps, futs)):
        e, H = f.result()
        g, gx = oracle.problem_inputs(p)
        e0, _, _ = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        assert e == e0
        assert H.shape == (p.n_pert, p.n_pert)
    st = srv.stats()
    assert st["completed"] == 8 and st["p50_s"] is not None and st["p99_s"] >= st["p50_s"]


def test_requests_overlap_and_late_arrivals_are_admitted_while_others_run():
    ps = mols(6)
    ex = FakeExecutor(seconds_per_pair_pert=5e-8)
    srv = Server(ex, budget_bytes=10 ** 12, n_slots=4)
    reqs = [Request(k, f"m{k}", p) for k, p in enumerate(ps)]
    srv.submit(reqs[0], at=0.0)
    srv.submit(reqs[1], at=0.0)
    for k in range(2, 6):
        srv.submit(reqs[k], at=0.001 * k)
    srv.run_until_idle(timeout_s=60)
    assert ex.max_active >= 2
    # some request admitted after another was admitted but before it finished
    overlapped = any(b.admitted > a.admitted and b.admitted < a.finished
                     for a in reqs for b in reqs if a is not b)
    assert overlapped
    assert all(r.status == "done" for r in reqs)


def test_slots_limit_concurrency():
    ps = mols(6)
    ex = FakeExecutor(seconds_per_pair_pert=5e-8)
    srv = Server(ex, budget_bytes=10 ** 12, n_slots=2)
    for k, p in enumerate(ps):
        srv.submit(Request(k, f"m{k}", p), at=0.0)
    while srv.step():
        assert len(srv.running) <= 2
    assert ex.max_active <= 2


def test_oversized_request_rejected_others_run():
    ps = mols(4)
    ex = FakeExecutor(seconds_per_pair_pert=1e-9)
    sizes = [ex.footprint(p) for p in ps]
    big = int(np.argmax(sizes))
    budget = sorted(sizes)[-2]           # everything but the largest fits
    if sizes.count(max(sizes)) > 1:
        pytest.skip("tie in footprints")
    srv = Server(ex, budget, n_slots=2)
    futs = [srv.submit(Request(k, f"m{k}", p)) for k, p in enumerate(ps)]
    srv.run_until_idle(timeout_s=60)
    with pytest.raises(MemoryError):
        futs[big].result()
    for k, f in enumerate(futs):
        if k != big:
            f.result()
    assert srv.stats()["rejected"] == 1


def test_failure_is_isolated():
    ps = mols(4)
    ex = FakeExecutor(seconds_per_pair_pert=1e-9, fail_mol={"m2"})
    srv = Server(ex, budget_bytes=10 ** 12, n_slots=2)
    futs = [srv.submit(Request(k, f"m{k}", p)) for k, p in enumerate(ps)]
    srv.run_until_idle(timeout_s=60)
    with pytest.raises(RuntimeError):
        futs[2].result()
    for k in (0, 1, 3):
        futs[k].result()
    assert srv.stats()["failed"] == 1


class CountingExecutor(FakeExecutor):
    def __init__(self, **kw):
        super().__init__(**kw)
        self.loads = []
        self.releases = 0

    def load(self, mol_id, problem):
        self.loads.append(mol_id)
        return super().load(mol_id, problem)

    def release(self, state):
        self.releases += 1
        super().release(state)


def test_resident_state_reused_and_evicted_lru():
    ps = mols(3)
    ex = CountingExecutor(seconds_per_pair_pert=1e-9)
    fp = [ex.footprint(p) for p in ps]
    budget = fp[0] + max(fp[1], fp[2]) + 1     # room for m0 plus one of the others
    srv = Server(ex, budget, n_slots=1)
    order = ["m0", "m0", "m1", "m0", "m2", "m0"]
    idx = {"m0": 0, "m1": 1, "m2": 2}
    for k, m in enumerate(order):
        srv.submit(Request(k, m, ps[idx[m]]), at=0.0)
    srv.run_until_idle(timeout_s=60)
    assert ex.loads.count("m0") == 1           # m0 stays resident (recently used)
    assert ex.loads.count("m1") == 1 and ex.loads.count("m2") == 1
    assert ex.releases >= 1                    # m1 evicted to make room for m2
    assert srv.peak_used <= budget


def test_one_request_per_molecule_at_a_time():
    p = mols(1)[0]
    ex = FakeExecutor(seconds_per_pair_pert=2e-8)
    srv = Server(ex, budget_bytes=10 ** 12, n_slots=4)
    for k in range(4):
        srv.submit(Request(k, "same", p), at=0.0)
    while srv.step():
        assert sum(1 for r, _, _ in srv.running.values() if r.mol_id == "same") <= 1


def test_cancel_queued():
    ps = mols(3)
    ex = FakeExecutor(seconds_per_pair_pert=1e-7)
    srv = Server(ex, budget_bytes=10 ** 12, n_slots=1)
    futs = [srv.submit(Request(k, f"m{k}", p)) for k, p in enumerate(ps)]
    srv.step()                                 # admits request 0
    assert srv.cancel(2)
    srv.run_until_idle(timeout_s=60)
    assert futs[2].cancelled()
    futs[0].result()
    futs[1].result()


def test_background_thread_mode():
    ps = mols(3)
    ex = FakeExecutor(seconds_per_pair_pert=1e-9)
    srv = Server(ex, budget_bytes=10 ** 12, n_slots=2)
    srv.start()
    try:
        futs = [srv.submit(Request(k, f"m{k}", p)) for k, p in enumerate(ps)]
        for f in futs:
            f.result(timeout=60)
    finally:
        srv.stop()


def test_request_kinds_and_incremental_accounting():
    """Hessian, gradient and response requests on the same molecules: each
    result matches the oracle for its kind, and a response on a resident
    molecule is charged only its response workspace (once per n_t growth)."""
    import oracle
    ps = mols(2, seed=7)
    ex = FakeExecutor(seconds_per_pair_pert=1e-8)
    trial = {k: inputs.trial_densities(p, 3 + k, 40 + k) for k, p in enumerate(ps)}
    srv = Server(ex, 10 * max(ex.footprint(p) for p in ps), n_slots=2)
    plan = [(0, "hessian"), (1, "response"), (0, "response"), (1, "gradient"), (0, "response"),
            (1, "hessian")]
    futs = []
    for k, (m, kind) in enumerate(plan):
        req = Request(k, f"m{m}", ps[m], kind=kind, trial=trial[m] if kind == "response" else None)
        futs.append((req, srv.submit(req, at=0.001 * k)))
    srv.run_until_idle(timeout_s=60)
    for (req, f), (m, kind) in zip(futs, plan):
        p = ps[m]
        g, gx = oracle.problem_inputs(p)
        if kind == "response":
            fr, fg = f.result()
            rt, gt = trial[m]
            Yr, Yg = oracle.response_rows(0, p.n_grid, p.coords, p.weights, p.rho, g, p.b, p.C, rt,
                                          oracle.gamma_x(p.grad_rho, gt))
            assert np.array_equal(fr, Yr) and np.array_equal(fg, Yg)
            assert req.pair_pert == float(p.n_grid) ** 2 * rt.shape[0]
        elif kind == "gradient":
            e, G = f.result()
            G0 = oracle.gradient(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                 p.rho_x, gx)
            assert np.array_equal(G, G0)
        else:
            e, H = f.result()
            assert H.shape == (p.n_pert, p.n_pert)
    # each molecule: base state plus one response workspace, charged once
    for m, p in enumerate(ps):
        base = ex.footprint(p)
        resp = ex.footprint(Request(0, "", p, kind="response", trial=trial[m])) - base
        assert srv.resident[f"m{m}"][0] == base + resp
    assert srv.used == sum(b for b, _ in srv.resident.values())
    srv.close()
