"""Continuous-batching server for VV10 Hessian-term requests.

A request names a molecule (grid, density and perturbed densities) and asks
for its energy and Hessian terms (kind "hessian"), its energy and nuclear
gradient ("gradient"), or the orbital-Hessian response of n_t trial
densities ("response", the step a CPSCF or TDDFT iteration repeats on a
resident grid).  The scheduler keeps up to `n_slots`
requests in flight at once, each on its own HIP stream, and admits a
waiting request as soon as a slot is free AND its device footprint fits in
what is left of the HBM budget; requests that arrive while others run are
admitted as slots and memory free up, so their work overlaps on the device.
Admission is first-come first-served, except that a request that does not
fit may be overtaken by later ones that do (bounded by `max_bypass`, after
which the head of the queue waits for memory).  A request larger than the
whole budget is rejected.

Device state of a molecule (its plan, inputs and workspace) stays resident
after its request completes, keyed by molecule id, and is reused by later
requests for the same molecule; idle resident state is evicted least
recently used when the budget needs room.  A request of another kind on a
resident molecule is charged only the memory its kind adds (for instance
the response workspace for its n_t).

The scheduler is independent of the device: `GpuExecutor` runs requests
through the HIP library; the CPU tests drive it with an executor of their
own (same interface: footprint, extra_bytes, load, start, poll, result,
release).
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future


@dataclasses.dataclass
class Request:
    rid: int
    mol_id: str
    problem: object                 # inputs.Problem with derivatives
    kind: str = "hessian"           # hessian, gradient or response
    trial: tuple = None             # response: (rho_t [n_t, N], grad_rho_t [n_t, N, 3])
    arrival: float = 0.0            # seconds on the server clock
    # filled by the server
    admitted: float = None
    finished: float = None
    status: str = "queued"          # queued, running, done, failed, rejected, cancelled
    error: str = None

    @property
    def n_cols(self) -> int:
        return int(self.trial[0].shape[0]) if self.kind == "response" else self.problem.n_pert

    @property
    def pair_pert(self) -> float:
        n = float(self.problem.n_grid)
        return n * n * self.n_cols

    @property
    def latency(self) -> float:
        return None if self.finished is None else self.finished - self.arrival


def as_request(x) -> Request:
    """A Request as given, or a Hessian request for a bare problem."""
    return x if isinstance(x, Request) else Request(rid=-1, mol_id="", problem=x)


def percentile(values, q):
    if not values:
        return None
    v = sorted(values)
    k = (len(v) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


class Server:
    """Scheduler core.  Drive it either with `run_until_idle()` (single
    thread, arrivals pre-scheduled) or with `start()` / `submit()` from other
    threads."""

    def __init__(self, executor, budget_bytes: int, n_slots: int = 4, max_bypass: int = 8,
                 clock=time.monotonic):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.n_slots = int(n_slots)
        self.max_bypass = int(max_bypass)
        self.clock = clock
        self.t0 = clock()
        self.queue = collections.deque()
        self.pending = []               # (arrival, request, future) not yet arrived
        self.running = {}               # slot -> (request, handle, future)
        self.resident = collections.OrderedDict()   # mol_id -> (bytes, state), LRU order
        self.pinned = collections.Counter()         # mol_id -> running requests using it
        self.used = 0
        self.peak_used = 0
        self.done = []
        self.lock = threading.Lock()
        self.bypassed = 0
        self._thread = None
        self._stop = False

    # -- time ------------------------------------------------------------
    def now(self) -> float:
        return self.clock() - self.t0

    # -- submission --------------------------------------------------------
    def submit(self, req: Request, at: float = None) -> Future:
        """Queue a request (at server time `at`, default now)."""
        fut = Future()
        with self.lock:
            if at is None or at <= self.now():
                req.arrival = self.now() if at is None else at
                self.queue.append((req, fut))
            else:
                req.arrival = at
                self.pending.append((at, req, fut))
                self.pending.sort(key=lambda x: x[0])
        return fut

    def cancel(self, rid: int) -> bool:
        with self.lock:
            for k, (req, fut) in enumerate(self.queue):
                if req.rid == rid:
                    del self.queue[k]
                    req.status = "cancelled"
                    fut.cancel()
                    return True
        return False

    # -- memory ------------------------------------------------------------
    def _footprint(self, req) -> int:
        """Bytes this request adds: its molecule's whole state, or what its kind
        adds to the resident state."""
        if req.mol_id in self.resident:
            return self.ex.extra_bytes(self.resident[req.mol_id][1], req)
        return self.ex.footprint(req)

    def _make_room(self, need: int) -> bool:
        """Evict idle resident molecules (LRU) until `need` bytes fit."""
        while self.used + need > self.budget:
            victim = next((m for m in self.resident if self.pinned[m] == 0), None)
            if victim is None:
                return False
            nbytes, state = self.resident.pop(victim)
            self.ex.release(state)
            self.used -= nbytes
        return True

    def _admit_one(self) -> bool:
        free = [s for s in range(self.n_slots) if s not in self.running]
        if not free or not self.queue:
            return False
        for k, (req, fut) in enumerate(self.queue):
            if k > 0 and self.bypassed >= self.max_bypass:
                break
            if self.pinned[req.mol_id] > 0:
                continue                    # one request per molecule at a time (shared state)
            total = self.ex.footprint(req)
            if total > self.budget:
                del self.queue[k]
                req.status = "rejected"
                req.error = f"footprint {total} bytes exceeds the budget {self.budget}"
                req.finished = self.now()
                self.done.append(req)
                fut.set_exception(MemoryError(req.error))
                return True
            need = self._footprint(req)
            if not self._make_room(need):
                continue
            del self.queue[k]
            self.bypassed = self.bypassed + 1 if k > 0 else 0
            slot = free[0]
            try:
                if req.mol_id in self.resident:
                    nbytes, state = self.resident.pop(req.mol_id)
                    self.resident[req.mol_id] = (nbytes + need, state)   # most recently used
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                else:
                    state = self.ex.load(req.mol_id, req.problem)
                    self.resident[req.mol_id] = (need, state)
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                self.pinned[req.mol_id] += 1
                handle = self.ex.start(state, req, slot)
            except Exception as e:          # the request fails; the server goes on
                self.pinned[req.mol_id] -= 1 if self.pinned[req.mol_id] > 0 else 0
                req.status, req.error, req.finished = "failed", repr(e), self.now()
                self.done.append(req)
                fut.set_exception(e)
                return True
            req.admitted = self.now()
            req.status = "running"
            self.running[slot] = (req, handle, fut)
            return True
        return False

    def _reap(self) -> int:
        n = 0
        for slot in list(self.running):
            req, handle, fut = self.running[slot]
            try:
                ready = self.ex.poll(handle)
                if not ready:
                    continue
                result = self.ex.result(handle)
                req.status = "done"
                fut.set_result(result)
            except Exception as e:
                req.status, req.error = "failed", repr(e)
                fut.set_exception(e)
            req.finished = self.now()
            self.pinned[req.mol_id] -= 1
            del self.running[slot]
            self.done.append(req)
            n += 1
        return n

    def step(self) -> bool:
        """One scheduling round; returns True while work remains."""
        with self.lock:
            now = self.now()
            while self.pending and self.pending[0][0] <= now:
                _, req, fut = self.pending.pop(0)
                self.queue.append((req, fut))
            self._reap()
            while self._admit_one():
                pass
            return bool(self.queue or self.running or self.pending)

    def run_until_idle(self, poll_s: float = 2e-4, timeout_s: float = None):
        start = self.clock()
        while self.step():
            if timeout_s is not None and self.clock() - start > timeout_s:
                raise TimeoutError("server did not drain")
            time.sleep(poll_s)

    # -- background mode ------------------------------------------------------
    def start(self, poll_s: float = 2e-4):
        def loop():
            while not self._stop:
                if not self.step():
                    time.sleep(poll_s * 5)
                else:
                    time.sleep(poll_s)
        self._thread = threading.Thread(target=loop, daemon=True)
        self._thread.start()

    def stop(self):
        self._stop = True
        if self._thread:
            self._thread.join()

    def close(self):
        with self.lock:
            for _, (nbytes, state) in self.resident.items():
                self.ex.release(state)
            self.resident.clear()
            self.used = 0

    # -- statistics ------------------------------------------------------------
    def stats(self, skip: int = 0) -> dict:
        reqs = sorted((r for r in self.done if r.status == "done"), key=lambda r: r.rid)[skip:]
        lat = [r.latency for r in reqs]
        if not reqs:
            return {"completed": 0}
        t_first = min(r.arrival for r in reqs)
        t_last = max(r.finished for r in reqs)
        work = sum(r.pair_pert for r in reqs)
        return {
            "completed": len(reqs),
            "failed": sum(1 for r in self.done if r.status == "failed"),
            "rejected": sum(1 for r in self.done if r.status == "rejected"),
            "p50_s": percentile(lat, 50),
            "p99_s": percentile(lat, 99),
            "mean_s": sum(lat) / len(lat),
            "throughput_pair_pert_per_s": work / (t_last - t_first) if t_last > t_first else None,
            "peak_bytes": self.peak_used,
            "budget_bytes": self.budget,
        }


class GpuExecutor:
    """Runs requests through the HIP library, one HIP stream per slot."""

    def __init__(self, prec: str = "bf16x3", n_slots: int = 4, device: str = "cuda", tiles="auto"):
        import torch
        from . import vv10
        self.torch, self.vv10 = torch, vv10
        self.prec = prec
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_slots)]
        self.load_stream = torch.cuda.Stream(device=self.dev)   # uploads and preparation
        self.tiles = tiles

    def _resp_bytes(self, n, n_t) -> int:
        prec = self.vv10.PRECISIONS[self.prec]
        return self.vv10.vv10_response_footprint_bytes(n, n_t, prec) + 8 * n * n_t * (4 + 2)

    def _grad_bytes(self, n, na) -> int:
        return self.vv10.vv10_gradient_footprint_bytes(n, na)

    def footprint(self, req) -> int:
        """Device bytes of the molecule's state once it has served `req`: plan
        and workspace (upper bound), inputs, and for a gradient the gradient
        pass's buffers, for a response the response workspace, trial
        densities and outputs."""
        req = as_request(req)
        problem = req.problem
        n, na = int(problem.n_grid), int(problem.n_atom)
        inputs = 8 * n * (3 + 1 + 1 + 3) + 4 * n + 8 * 3 * na * n * 4
        b = self.vv10.vv10_footprint_bytes(n, na, self.vv10.PRECISIONS[self.prec]) + inputs
        if req.kind == "response":
            b += self._resp_bytes(n, req.n_cols)
        elif req.kind == "gradient":
            b += self._grad_bytes(n, na)
        return b

    def extra_bytes(self, state, req) -> int:
        """Bytes `req` adds to a resident state: a larger response workspace,
        or the gradient pass's buffers the first time the molecule serves a
        gradient."""
        n = int(req.problem.n_grid)
        if req.kind == "response":
            return max(0, self._resp_bytes(n, req.n_cols) - state.get("resp_bytes", 0))
        if req.kind == "gradient" and not state.get("grad_bytes"):
            return self._grad_bytes(n, int(req.problem.n_atom))
        return 0

    def load(self, mol_id, problem):
        torch = self.torch
        with torch.cuda.stream(self.load_stream):
            plan = self.vv10.Plan(problem, prec=self.prec, device=self.dev,
                                  stream=self.load_stream, tiles=self.tiles)
            rx = torch.as_tensor(problem.rho_x, dtype=torch.float64).to(self.dev).contiguous()
            gx = torch.as_tensor(problem.grad_rho_x, dtype=torch.float64).to(self.dev).contiguous()
        self.load_stream.synchronize()
        return {"plan": plan, "rx": rx, "gx": gx}

    def start(self, state, req, slot):
        torch, vv = self.torch, self.vv10
        s = self.streams[slot]
        plan = state["plan"]
        P = 3 * plan.n_atom
        # the plan's previous calls completed before this request was admitted
        # (one request per molecule at a time), so it can move to this slot
        vv.vv10_set_stream(plan.handle, s)
        out = {}
        if req.kind == "response":
            n = plan.n
            state["resp_bytes"] = max(state.get("resp_bytes", 0), self._resp_bytes(n, req.n_cols))
            with torch.cuda.stream(s):
                rt = torch.as_tensor(req.trial[0], dtype=torch.float64).to(self.dev, non_blocking=False).contiguous()
                gt = torch.as_tensor(req.trial[1], dtype=torch.float64).to(self.dev, non_blocking=False).contiguous()
                fr = torch.empty((req.n_cols, n), dtype=torch.float64, device=self.dev)
                fg = torch.empty_like(fr)
            vv.vv10_trial_response(plan.handle, req.n_cols, rt, gt, fr, fg)
            out.update(fr=fr, fg=fg, keep=(rt, gt))
        else:
            with torch.cuda.stream(s):
                e = torch.empty(1, dtype=torch.float64, device=self.dev)
                res = torch.empty((P, P) if req.kind == "hessian" else P, dtype=torch.float64,
                                  device=self.dev)
            if req.kind == "hessian":
                # energy and Hessian terms from one pass over the pairs
                vv.vv10_nuclear_terms(plan.handle, P, state["rx"], state["gx"], hess=res, energy=e)
            else:
                state["grad_bytes"] = self._grad_bytes(plan.n, plan.n_atom)
                vv.vv10_energy_potential(plan.handle, e)
                vv.vv10_gradient(plan.handle, P, state["rx"], state["gx"], res)
            out.update(e=e, res=res)
        done = torch.cuda.Event()
        done.record(s)
        out.update(done=done, kind=req.kind)
        return out

    def poll(self, handle) -> bool:
        return handle["done"].query()

    def result(self, handle):
        handle["done"].synchronize()
        if handle["kind"] == "response":
            return handle["fr"].cpu().numpy(), handle["fg"].cpu().numpy()
        return handle["e"].item(), handle["res"].cpu().numpy()

    def release(self, state):
        state["plan"].close()
        state.clear()

