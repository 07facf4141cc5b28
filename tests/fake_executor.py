"""CPU stand-in executor for the server's scheduler tests (test
infrastructure: results from the FP64 oracle, completion after a delay
proportional to N^2 P)."""
import time

import oracle
from paper_2208_14639_amd.serve import as_request


class FakeExecutor:
    """CPU stand-in: results from the FP64 oracle, completion after
    `seconds_per_pair_pert * N^2 P` of wall time, footprint from the same
    formula the library uses, optional injected failures."""

    def __init__(self, seconds_per_pair_pert: float = 1e-9, fail_mol=None, clock=time.monotonic):
        self.spp = seconds_per_pair_pert
        self.fail_mol = set(fail_mol or ())
        self.clock = clock
        self.active = 0
        self.max_active = 0

    def footprint(self, req) -> int:
        req = as_request(req)
        n, na = int(req.problem.n_grid), int(req.problem.n_atom)
        b = 8 * n * (20 + 8 * 3 * na)
        if req.kind == "response":
            b += 8 * n * 10 * req.n_cols
        return b

    def extra_bytes(self, state, req) -> int:
        if req.kind != "response":
            return 0
        return max(0, 8 * int(req.problem.n_grid) * 10 * req.n_cols - state.get("resp_bytes", 0))

    def load(self, mol_id, problem):
        if mol_id in self.fail_mol:
            raise RuntimeError(f"injected load failure for {mol_id}")
        return {"mol": mol_id}

    def start(self, state, req, slot):
        problem = req.problem
        g, gx = oracle.problem_inputs(problem)
        if req.kind == "response":
            state["resp_bytes"] = max(state.get("resp_bytes", 0),
                                      8 * int(problem.n_grid) * 10 * req.n_cols)
            rt, gt = req.trial
            res = oracle.response_rows(0, problem.n_grid, problem.coords, problem.weights,
                                       problem.rho, g, problem.b, problem.C, rt,
                                       oracle.gamma_x(problem.grad_rho, gt))
        else:
            e, _, _ = oracle.energy_potential(problem.coords, problem.weights, problem.rho, g,
                                              problem.b, problem.C)
            if req.kind == "hessian":
                H, _ = oracle.hessian_terms(problem.atom_of, problem.n_atom, problem.coords,
                                            problem.weights, problem.rho, g, problem.b, problem.C,
                                            problem.rho_x, gx)
            else:
                H = oracle.gradient(problem.atom_of, problem.n_atom, problem.coords,
                                    problem.weights, problem.rho, g, problem.b, problem.C,
                                    problem.rho_x, gx)
            res = (e, H)
        n = float(problem.n_grid)
        self.active += 1
        self.max_active = max(self.max_active, self.active)
        return {"t_done": self.clock() + self.spp * n * n * req.n_cols, "res": res}

    def poll(self, handle) -> bool:
        ready = self.clock() >= handle["t_done"]
        if ready and not handle.get("counted"):
            handle["counted"] = True
            self.active -= 1
        return ready

    def result(self, handle):
        return handle["res"]

    def release(self, state):
        state.clear()
