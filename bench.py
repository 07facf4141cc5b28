#!/usr/bin/env python3
"""Benchmark of the VV10 Hessian-term engine on one MI355X.

Default run: the water 20-mer (N = 120000 grid points, P = 180 nuclear
perturbations).  One step is one pass of the whole hot path over the
molecule, already resident in HBM: vv10_prepare (per-point prep) ->
vv10_nuclear_terms with the energy, potential, Hessian-term and gradient
outputs (one pass over the pairs for the pair integrals and the
grid-position terms, potential and energy, perturbation packing, MFMA
contraction, assembly) -> vv10_destroy.  The split-BF16 path is timed, then
the FP64 and FP32 paths on the same inputs ("mixed vs FP64"), and the run
reports:
  * every mixed output against the FP64 GPU path element by element
    (energy, potential, gradient, every Hessian element, response rows);
  * every path against the FP64 oracle on rows sampled at three places
    (potential and response rows of 4 points each);
  * a served stream (continuous batching, Poisson arrivals, a fresh seeded
    cluster per request) with p50/p99 latency, each result checked against
    the FP64 GPU path alone and the smallest against the oracle;
  * the oracle timed on the host cores on a bounded row sample.
--separate-energy times vv10_energy_potential (its own pair pass) followed
by vv10_hessian_terms instead.

Metric: grid-pair x perturbation per second, N^2 P / t_step, with N^2 the
ordered pairs (self pairs included) and P = 3 N_atom.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (the perturbation contraction, timed with HIP events recorded by the
library on the plan's stream), the pair pass against the vector peak, the
comparison legs with their errors, the served latencies and a CPU baseline
(rank 0 only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS_TFLOPS = {"mfma_f64": 78.6, "mfma_f32": 157.3, "mfma_bf16": 2500.0, "valu_f32": 157.3,
                "valu_f64": 78.6}
HBM_GBS = 8000.0
# algorithmic work per unit, counted from the formulas (FMA = 2 flops)
FLOPS_PER_PAIR_PERT = 8          # contraction: 4 FMAs per pair and perturbation
FLOPS_PER_PAIR_PERT_W = 6        # weight contraction: 3 FMAs per pair and perturbation
FLOPS_PER_PAIR_INTEGRALS = 38    # E, U, W (26) + A, B, C (12)
FLOPS_PER_PAIR_EUW = 26          # k_pair, energy call: E, U, W
# fused grid pass (k_grid with the pair integrals), per pair by atom class:
# the outer point's own atom (pair geometry 22 + six integral sums 14), an
# atom B below it (+ the grid sums E^{Bgr} + c U^{Bgr} and W^{Bgr}, 29), an atom above
# it (+ E^{Bgr}, U^{Bgr} and W^{Bgr} apart, 34, and the D sums, 24)
FLOPS_GRID_OWN, FLOPS_GRID_BELOW, FLOPS_GRID_ABOVE = 36, 65, 94
FP32_NO_PACKED_TFLOPS = 78.6     # one FP32 FMA per lane and cycle (packed FP32 off)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
METRIC = "VV10 Hessian grid-pair\u00b7perturbation/s, mixed vs FP64, at stated err; p99 latency"
DTYPES = {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f32+f64"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src):
    """C/C++/HIP source without its comments and with runs of white space
    collapsed: an edit of a comment leaves it unchanged, any edit of the code
    changes it (string and character literals are kept as written)."""
    out, code, i, n = [], [], 0, len(src)

    def flush():
        out.extend("".join(code).split())
        code.clear()

    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            flush()
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            code.append(" ")
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            code.append(" ")
            i = n if j < 0 else j + 2
        else:
            code.append(c)
            i += 1
    flush()
    return " ".join(out)


def source_sha(rels):
    """Hash of the code (not the comments) of the source files that a
    counter record was taken from."""
    h = hashlib.sha256()
    for rel in rels:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def counter_record(kernel_key, workload, prec):
    """The committed rocprofv3 counter summary of a kernel (HBM bytes per
    launch, VALU-issue and MFMA busy fractions), or None when the kernel
    source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(f"{kernel_key}:{workload}:{prec}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_sha(rec["sources"]):
        return None
    return rec


def measured_traffic(kernel_key, workload, prec):
    rec = counter_record(kernel_key, workload, prec)
    return None if rec is None else rec["bytes_per_launch"]


def pair_pass_roofline(p, kernel, ms, prec):
    """Algorithmic FP32 (FP64) VALU rate of the pair pass against the vector
    peak; the FP32 peak counts packed FP32 (two FMAs per lane and cycle),
    which all device code here is built without, so the rate is also given
    against one FMA per lane and cycle."""
    import numpy as np
    cnt = np.bincount(p.atom_of, minlength=p.n_atom).astype(np.float64)
    n = float(p.n_grid)
    if kernel == "k_pair":
        flops = FLOPS_PER_PAIR_EUW * n * n
    else:
        own = float(np.sum(cnt * cnt))
        cross = (n * n - own) / 2.0               # pairs with B above (= below) the outer atom
        flops = FLOPS_GRID_OWN * own + (FLOPS_GRID_BELOW + FLOPS_GRID_ABOVE) * cross
    achieved = flops / (ms * 1e-3) / 1e12
    peak = PEAKS_TFLOPS["valu_f64" if prec == "fp64" else "valu_f32"]
    out = dict(bound="alu", kernel=kernel, achieved=achieved, peak=peak, unit="TFLOP/s",
               frac=achieved / peak, flops_per_pair=flops / (n * n))
    if prec != "fp64":
        out["peak_no_packed"] = FP32_NO_PACKED_TFLOPS
        out["frac_no_packed"] = achieved / FP32_NO_PACKED_TFLOPS
    return out


def row_sample(fn, n, target_s=10.0):
    """Rows 0..k of a row-wise oracle step fn(k), k sized so that the timed
    call takes about target_s.  Each call has a fixed cost (a full
    pair-integral pass) besides its per-row cost, so k grows by 4x until a
    call takes a quarter of the target, and the last two calls give the
    linear model used to size the timed call.  Returns (k, seconds, result)."""
    k, prev = min(n, 256), None
    while True:
        t0 = time.perf_counter()
        res = fn(k)
        t = time.perf_counter() - t0
        if k >= n or t >= target_s / 4:
            break
        prev = (k, t)
        k = min(n, 4 * k)
    if prev is not None and k > prev[0] and t > prev[1]:
        per = (t - prev[1]) / (k - prev[0])
        fixed = max(t - per * k, 0.0)
    else:
        per, fixed = t / k, 0.0
    k2 = int(max(16, min(n, (target_s - fixed) / per)))
    if k2 <= k:
        return k, t, res
    t0 = time.perf_counter()
    res = fn(k2)
    return k2, time.perf_counter() - t0, res


def host_info():
    """Provenance of a host-side timing: CPU model, logical CPUs visible to
    the process and the OpenMP thread setting."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(p, budget_s=30.0):
    """FP64 oracle on the host.  Full workload when it fits the budget, else
    the dominant O(N^2 P) step (response rows, and with weight derivatives the
    weight integrals of the same rows) on a row sample."""
    import oracle
    g, gx = oracle.problem_inputs(p)
    n, P = p.n_grid, p.n_pert
    est_rate = 3e9 * oracle.num_threads() / 8      # pair*pert/s, measured order of magnitude
    base = dict(unit="pair*pert/s", cores=oracle.num_threads(), kind="oracle", **host_info())
    if p.w_x is not None:
        def rows(k):
            oracle.response_rows(0, k, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
            oracle.weight_integrals(p.coords, p.rho, g, p.b, p.C, p.w_x, 0, k)
        k, dt, _ = row_sample(rows, n)
        return dict(value=k * n * P / dt, seconds=dt,
                    sample=f"response rows and weight integrals of rows 0..{k} of N={n}, P={P} "
                           f"(the dominant N^2 P steps)", **base), None
    if n * n * P / est_rate <= budget_s:
        t0 = time.perf_counter()
        H, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                    p.rho_x, gx)
        e0, fr0, fg0 = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        dt = time.perf_counter() - t0
        return dict(value=n * n * P / dt, seconds=dt,
                    sample=f"whole workload: energy, potential and Hessian terms, N={n}, P={P}",
                    **base), dict(H=H, E=e0, f_rho=fr0, f_gamma=fg0)
    k, dt, _ = row_sample(
        lambda k: oracle.response_rows(0, k, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx), n)
    return dict(value=k * n * P / dt, seconds=dt,
                sample=f"response rows 0..{k} of N={n}, P={P} (the dominant N^2 P step: each "
                       f"row sums over all N points for all P perturbations)", **base), None


ROW_SAMPLE = 4          # rows per sampled place


def sample_places(n):
    """Three places of ROW_SAMPLE rows: the first points, the middle, the last."""
    mid = n // 2 + 7
    return [0, min(mid, n - ROW_SAMPLE), n - ROW_SAMPLE]


def oracle_row_checks(p, results):
    """Potential (f^rho, f^gamma) and response rows of the oracle on rows
    sampled at three places, against each path's GPU outputs (normwise over
    the sampled rows, scaled by the largest GPU value of the whole output).
    results: {prec: dict(f_rho, f_gamma, resp_rho, resp_gamma)} as numpy."""
    import numpy as np
    import oracle
    g, gx = oracle.problem_inputs(p)
    places = sample_places(p.n_grid)
    ref = []
    for i0 in places:
        fr, fg, _ = oracle.potential_rows(i0, i0 + ROW_SAMPLE, p.coords, p.weights, p.rho, g, p.b, p.C)
        Yr, Yg = oracle.response_rows(i0, i0 + ROW_SAMPLE, p.coords, p.weights, p.rho, g, p.b, p.C,
                                      p.rho_x, gx)
        ref.append((i0, fr, fg, Yr, Yg))
    out = {"rows": [[i0, i0 + ROW_SAMPLE] for i0 in places]}
    for prec, r in results.items():
        e = dict(f_rho=0.0, f_gamma=0.0, resp_rho=0.0, resp_gamma=0.0)
        scale = {k: float(np.max(np.abs(r[k]))) for k in e}
        for i0, fr, fg, Yr, Yg in ref:
            sl = slice(i0, i0 + ROW_SAMPLE)
            e["f_rho"] = max(e["f_rho"], float(np.max(np.abs(r["f_rho"][sl] - fr))) / scale["f_rho"])
            e["f_gamma"] = max(e["f_gamma"], float(np.max(np.abs(r["f_gamma"][sl] - fg))) / scale["f_gamma"])
            e["resp_rho"] = max(e["resp_rho"], float(np.max(np.abs(r["resp_rho"][:, sl] - Yr))) / scale["resp_rho"])
            e["resp_gamma"] = max(e["resp_gamma"], float(np.max(np.abs(r["resp_gamma"][:, sl] - Yg))) / scale["resp_gamma"])
        out[prec] = e
    return out


def errors_vs(a, b):
    """Outputs a of one path against b of another (numpy dicts): energy
    relative; potential, gradient and response rows normwise; every Hessian
    element absolute (max and how many exceed the 1e-5 au bound)."""
    import numpy as np
    nw = lambda x, y: float(np.max(np.abs(x - y)) / np.max(np.abs(y)))
    out = {"energy_rel": abs(a["energy"] - b["energy"]) / abs(b["energy"]),
           "f_rho_normwise": nw(a["f_rho"], b["f_rho"]),
           "f_gamma_normwise": nw(a["f_gamma"], b["f_gamma"]),
           "grad_normwise": nw(a["grad"], b["grad"]),
           "hess_max_abs": float(np.max(np.abs(a["hess"] - b["hess"]))),
           "hess_elements_over_1e-5": int(np.sum(np.abs(a["hess"] - b["hess"]) > 1e-5)),
           "hess_elements": int(a["hess"].size),
           "hess_max_abs_value": float(np.max(np.abs(b["hess"])))}
    if "resp_rho" in a and "resp_rho" in b:
        out["resp_rho_normwise"] = nw(a["resp_rho"], b["resp_rho"])
        out["resp_gamma_normwise"] = nw(a["resp_gamma"], b["resp_gamma"])
    return out


def bench_batch(args, torch, np, inputs, vv10):
    """64 molecules of uneven size in one graph launch per step.  Every
    molecule's energy and Hessian terms are checked against the same batch
    run on the FP64 path; the oracle checks the three smallest molecules in
    full and the largest molecule's energy and sampled potential rows."""
    sizes = inputs.random_cluster_sizes(64, seed=1004)
    probs = []
    for m, k in enumerate(sizes):
        probs.append(inputs.make_problem(k, 1500, 2000 + m))
        if (m + 1) % 8 == 0:
            log(f"generated {m + 1}/64 molecules")
    pair_pert = float(sum(float(p.n_grid) ** 2 * p.n_pert for p in probs))
    log(f"batch: {sum(p.n_grid for p in probs)} points, {pair_pert:.3e} pair*pert")
    with vv10.Batch(probs, prec=args.prec, tiles="auto") as b:
        for k in range(args.warmup):
            b.run()
            torch.cuda.synchronize()
            log(f"warmup {k + 1}/{args.warmup} done")
        t0 = time.perf_counter()
        for k in range(args.steps):
            b.run()
            torch.cuda.synchronize()
            log(f"step {k + 1}/{args.steps} done")
        dt = (time.perf_counter() - t0) / args.steps
        n_items, n_wg = b.info()
        energies = b.energy.cpu().numpy()
        blocks = [h.cpu().numpy() for h in b.blocks()]
    out = {
        "metric": METRIC,
        "value": pair_pert / dt, "unit": "pair*pert/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.prec],
        "data": "synthetic",
        "config": {"workload": "batch64", "n_mol": len(probs), "waters": sizes, "n_pa": 1500,
                   "precision": args.prec, "work_items": n_items, "persistent_workgroups": n_wg},
        "roofline": None, "cpu_baseline": None,
    }
    # every molecule against the FP64 path (the same batch, one untimed launch;
    # --compare none skips it, e.g. for a kernel profile of the timed path alone)
    if args.prec != "fp64" and args.compare != "none":
        with vv10.Batch(probs, prec="fp64", tiles="auto") as b:
            t0 = time.perf_counter()
            b.run()
            torch.cuda.synchronize()
            t64 = time.perf_counter() - t0
            e64 = b.energy.cpu().numpy()
            H64 = [h.cpu().numpy() for h in b.blocks()]
        log("fp64 batch done")
        per = [{"mol": m, "n_grid": probs[m].n_grid,
                "energy_rel": float(abs(energies[m] - e64[m]) / abs(e64[m])),
                "hess_max_abs": float(np.max(np.abs(blocks[m] - H64[m])))} for m in range(len(probs))]
        out["vs_fp64"] = {"ms_per_launch": t64 * 1e3, "speedup_vs_one_fp64_launch": t64 / dt,
                          "energy_rel_max": max(r["energy_rel"] for r in per),
                          "hess_max_abs_max": max(r["hess_max_abs"] for r in per),
                          "within_stated_bounds": all(r["energy_rel"] <= 1e-6 and r["hess_max_abs"] <= 1e-5
                                                      for r in per),
                          "per_molecule": per}
    # CPU baseline: the whole oracle on the three smallest molecules, whose
    # results also check the batch's; the largest molecule's energy and
    # potential rows against the oracle
    if not args.no_cpu_baseline:
        import oracle
        order = np.argsort([p.n_grid for p in probs])
        errs = []
        work, secs = 0.0, 0.0
        for m in order[:3]:
            p = probs[m]
            g, gx = oracle.problem_inputs(p)
            t0 = time.perf_counter()
            H0, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g,
                                         p.b, p.C, p.rho_x, gx)
            e0, _, _ = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
            secs += time.perf_counter() - t0
            work += float(p.n_grid) ** 2 * p.n_pert
            errs.append({"mol": int(m), "n_grid": p.n_grid,
                         "energy_rel": abs(energies[m] - e0) / abs(e0),
                         "hess_max_abs": float(np.max(np.abs(blocks[m] - H0)))})
        big = int(order[-1])
        p = probs[big]
        log(f"oracle energy of the largest molecule (N={p.n_grid}) running ...")
        g = oracle.gamma(p.grad_rho)
        e0, _, _ = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        rec = {"mol": big, "n_grid": p.n_grid, "energy_rel": abs(energies[big] - e0) / abs(e0)}
        if args.prec != "fp64":
            rec["fp64_energy_rel"] = abs(e64[big] - e0) / abs(e0)
        errs.append(rec)
        out["cpu_baseline"] = dict(value=work / secs, unit="pair*pert/s", cores=oracle.num_threads(),
                                   kind="oracle", seconds=secs, **host_info(),
                                   sample="energy, potential and Hessian terms of the three "
                                          "smallest molecules of the batch")
        out["errors_vs_oracle"] = errs
    print(json.dumps(out), flush=True)


def bench_gradient(args, torch, np, inputs, vv10):
    """Geometry-optimisation step on the hexamer: prepare, energy/potential and
    the nuclear gradient alone (vv10_gradient), then destroy."""
    p = inputs.make_workload("water_hexamer")
    n, na, P = p.n_grid, p.n_atom, p.n_pert
    dev = torch.device("cuda:0")
    f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
    coords, w, rho, grad = f64(p.coords), f64(p.weights), f64(p.rho), f64(p.grad_rho)
    atom_of = torch.as_tensor(p.atom_of, dtype=torch.int32).to(dev).contiguous()
    rho_x, grad_x = f64(p.rho_x), f64(p.grad_rho_x)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    gradient = torch.empty(P, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    prec = vv10.PRECISIONS[args.prec]

    def step():
        h = vv10.vv10_prepare(p.b, p.C, n, na, coords, w, atom_of, rho, grad, prec, stream)
        try:
            vv10.vv10_set_timing(h, True)
            vv10.vv10_energy_potential(h, energy, None, None)
            vv10.vv10_gradient(h, P, rho_x, grad_x, gradient)
            st = vv10.vv10_stage_times(h)
        finally:
            vv10.vv10_destroy(h)
        return st

    for k in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        stages.append(step())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    stage_ms = {k: float(np.mean([st[k] for st in stages])) for k in ("pair", "grid", "potential", "assemble")}
    out = {
        "metric": "VV10 Hessian grid-pair\u00b7perturbation/s, mixed vs FP64, at stated err; p99 latency",
        "value": float(n) * n * P / dt, "unit": "pair*pert/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "f32+f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "gradient_hexamer", "n_grid": n, "n_atom": na, "n_pert": P,
                   "precision": args.prec, "seed": p.seed},
        "roofline": None,
        "stage_ms": stage_ms,
        "grad_pass_pairs_per_s": float(n) * n / (stage_ms["grid"] * 1e-3),
    }
    if not args.no_cpu_baseline:
        import oracle
        g, gx = oracle.problem_inputs(p)
        t0 = time.perf_counter()
        G0 = oracle.gradient(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
        e0, _, _ = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=float(n) * n * P / dtc, unit="pair*pert/s",
                                   cores=oracle.num_threads(), kind="oracle", seconds=dtc,
                                   sample=f"whole workload: energy, potential and gradient, N={n}")
        Gg = gradient.cpu().numpy()
        out["errors_vs_oracle"] = {"energy_rel": abs(energy.item() - e0) / abs(e0),
                                   "grad_normwise": float(np.max(np.abs(Gg - G0)) / np.max(np.abs(G0)))}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_trial_response(args, torch, np, inputs, vv10, n_t=54):
    """CPSCF-style use of vv10_trial_response: the hexamer plan is prepared
    once, and every step evaluates f^{rho,t}, f^{gamma,t} of n_t seeded trial
    densities on it (the first call also forms the pair integrals the plan
    then keeps; it is timed separately)."""
    p = inputs.make_workload("water_hexamer", with_derivatives=False)
    n = p.n_grid
    rt, gt = inputs.trial_densities(p, n_t, seed=1006)
    dev = torch.device("cuda:0")
    rt_d = torch.as_tensor(rt).to(dev).contiguous()
    gt_d = torch.as_tensor(gt).to(dev).contiguous()
    pair_t = float(n) * n * n_t
    with vv10.Plan(p, prec=args.prec) as pl:
        vv10.vv10_set_timing(pl.handle, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fr, fg = pl.trial_response(rt_d, gt_d)
        torch.cuda.synchronize()
        first_ms = (time.perf_counter() - t0) * 1e3
        first_stages = vv10.vv10_stage_times(pl.handle)
        for k in range(args.warmup):
            pl.trial_response(rt_d, gt_d)
        torch.cuda.synchronize()
        stages = []
        t0 = time.perf_counter()
        for k in range(args.steps):
            fr, fg = pl.trial_response(rt_d, gt_d)
            stages.append(vv10.vv10_stage_times(pl.handle))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        stage_ms = {k: float(np.mean([st[k] for st in stages])) for k in ("pert_prep", "contract", "assemble")}
        fr, fg = fr.cpu().numpy(), fg.cpu().numpy()
    t_con = stage_ms["contract"] * 1e-3
    mfma_key = {"fp64": "mfma_f64", "fp32": "mfma_f32", "bf16x3": "mfma_bf16"}[args.prec]
    achieved = FLOPS_PER_PAIR_PERT * pair_t / t_con / 1e12
    out = {
        "metric": "VV10 Hessian grid-pair\u00b7perturbation/s, mixed vs FP64, at stated err; p99 latency",
        "value": pair_t / dt, "unit": "pair*pert/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f32+f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "trial_response_hexamer", "n_grid": n, "n_trial": n_t,
                   "precision": args.prec, "seed": 1006},
        "roofline": dict(bound="mfma", kernel=f"k_contract_{args.prec}", achieved=achieved,
                         peak=PEAKS_TFLOPS[mfma_key], unit="TFLOP/s",
                         frac=achieved / PEAKS_TFLOPS[mfma_key], traffic=None),
        "stage_ms": stage_ms,
        "first_call_ms": first_ms, "first_call_pair_ms": first_stages["pair"],
    }
    if not args.no_cpu_baseline:
        import oracle
        g = oracle.gamma(p.grad_rho)
        gam_t = oracle.gamma_x(p.grad_rho, gt)
        # rows 0..k of the oracle's response (one pair-integral pass per call),
        # k sized to about 10 s
        k, dtc, (Yr, Yg) = row_sample(
            lambda k: oracle.response_rows(0, k, p.coords, p.weights, p.rho, g, p.b, p.C, rt, gam_t), n)
        err = max(float(np.max(np.abs(fr[:, :k] - Yr)) / np.max(np.abs(fr))),
                  float(np.max(np.abs(fg[:, :k] - Yg)) / np.max(np.abs(fg))))
        out["cpu_baseline"] = dict(value=k * n * n_t / dtc, unit="pair*pert/s",
                                   cores=oracle.num_threads(), kind="oracle", seconds=dtc,
                                   sample=f"response rows 0..{k} of N={n}, n_t={n_t} "
                                          f"(one full pair-integral pass included)")
        out["errors_vs_oracle"] = {"response_rows_0_to_k_normwise": err}
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def served_stream(args, torch, np, inputs, vv10, n_requests=56, n_warm=8, n_probe=8, load=0.7,
                  check=True):
    """Poisson stream of Hessian-term requests through the continuous-batching
    server, each a fresh seeded water cluster (1-30 waters, 1000-2500 points
    per atom, seed 3000 + k), its density and nuclear derivatives built on
    the device before the stream starts.  Arrival rate: `load` times the
    single-slot capacity measured on the first n_probe requests.  Returns
    the served record: p50/p99 latency (the first n_warm requests are
    warm-up), throughput, a latency breakdown by request size (queue wait
    and service time), and the result checks: every result against the same
    request run alone (bitwise) and alone on the FP64 path (stated bounds),
    and the two smallest requests against the oracle."""
    from paper_2208_14639_amd.serve import GpuExecutor, Request, Server, percentile
    rng = np.random.default_rng(1005)
    dev = torch.device("cuda:0")
    sizes = [(int(rng.integers(1, 31)), int(rng.integers(1000, 2501))) for _ in range(n_requests)]
    reqs_in = []
    for k, (nw, npa) in enumerate(sizes):
        reqs_in.append(inputs.make_problem_on_device(nw, npa, 3000 + k, torch, dev))
    torch.cuda.synchronize()
    log(f"served: {n_requests} requests built on the device "
        f"(N {min(q.n_grid for q in reqs_in)}..{max(q.n_grid for q in reqs_in)})")
    tiles = "auto"

    def alone(p, prec):
        with vv10.Plan(p, prec=prec, tiles=tiles) as pl:
            out = pl.nuclear_terms(p.rho_x, p.grad_rho_x, hess=True, energy=True)
            torch.cuda.synchronize()
            return out["energy"].item(), out["hess"].cpu().numpy()

    # single-slot service time (prepare + one Hessian-terms call) on the first
    # n_probe requests, after one untimed call each
    service = []
    for p in reqs_in[:n_probe]:
        alone(p, args.prec)
        t0 = time.perf_counter()
        alone(p, args.prec)
        service.append(time.perf_counter() - t0)
    rate = load / float(np.mean(service))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    ex = GpuExecutor(prec=args.prec, n_slots=4)
    budget = 96 * 1024 ** 3
    srv = Server(ex, budget, n_slots=4)
    futs = [srv.submit(Request(k, f"r{k}", reqs_in[k]), at=float(t))
            for k, t in enumerate(arrivals)]
    t0 = time.perf_counter()
    srv.run_until_idle(timeout_s=240)
    wall = time.perf_counter() - t0
    log(f"served: stream drained in {wall:.1f} s")
    st = srv.stats(skip=n_warm)
    done = sorted((r for r in srv.done if r.status == "done"), key=lambda r: r.rid)[n_warm:]
    # latency by request size: queue wait (arrival -> admission) and service
    buckets = [(0, 30000), (30000, 90000), (90000, 150000), (150000, 10 ** 9)]
    by_size = []
    for lo, hi in buckets:
        rs = [r for r in done if lo <= r.problem.n_grid < hi]
        if not rs:
            continue
        lat = [r.latency for r in rs]
        by_size.append({"n_grid": [lo, hi if hi < 10 ** 9 else None], "requests": len(rs),
                        "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
                        "mean_wait_s": float(np.mean([r.admitted - r.arrival for r in rs])),
                        "mean_service_s": float(np.mean([r.finished - r.admitted for r in rs]))})
    slow = sorted(done, key=lambda r: r.latency)[-3:]
    tail = [{"rid": r.rid, "n_grid": r.problem.n_grid, "n_pert": r.problem.n_pert,
             "latency_s": r.latency, "wait_s": r.admitted - r.arrival,
             "service_s": r.finished - r.admitted} for r in slow]
    rec = {"requests": n_requests, "warmup": n_warm, "reuse_fraction": 0.0,
           "request_sizes": "fresh cluster per request: U{1..30} waters, U{1000..2500} points/atom",
           "arrival_rate_per_s": rate, "rate_fraction_of_single_slot": load,
           "single_slot_mean_s": float(np.mean(service)), "slots": 4, "budget_bytes": budget,
           "wall_s": wall, "latency_s": {"p50": st["p50_s"], "p99": st["p99_s"], "mean": st["mean_s"]},
           "throughput_pair_pert_per_s": st["throughput_pair_pert_per_s"],
           "completed": st["completed"], "failed": st["failed"], "rejected": st["rejected"],
           "peak_bytes": st["peak_bytes"], "latency_by_size": by_size, "slowest": tail}
    if check:
        # every result against the same request alone (same precision,
        # bitwise) and alone on the FP64 path (stated bounds)
        same, e_max, h_max = True, 0.0, 0.0
        for k, f in enumerate(futs):
            e, H = f.result()
            ea, Ha = alone(reqs_in[k], args.prec)
            same &= bool(np.array_equal(H, Ha)) and e == ea
            e64, H64 = alone(reqs_in[k], "fp64")
            e_max = max(e_max, abs(e - e64) / abs(e64))
            h_max = max(h_max, float(np.max(np.abs(H - H64))))
        log("served: results checked against alone and FP64")
        rec["results_identical_alone_and_in_mix"] = same
        rec["vs_fp64_alone"] = {"energy_rel_max": e_max, "hess_max_abs_max": h_max,
                                "within_bounds": bool(e_max <= 1e-6 and h_max <= 1e-5)}
        import oracle
        chk = []
        for k in sorted(range(n_requests), key=lambda k: reqs_in[k].n_grid)[:2]:
            q = reqs_in[k]
            hp = inputs.Problem(mol=q.mol, atom_of=q.atom_of, offsets=q.offsets, coords=q.coords,
                                weights=q.weights, rho=q.rho.cpu().numpy(),
                                grad_rho=q.grad_rho.cpu().numpy(), radii=q.radii,
                                rho_x=q.rho_x.cpu().numpy(), grad_rho_x=q.grad_rho_x.cpu().numpy())
            g, gx = oracle.problem_inputs(hp)
            H0, _ = oracle.hessian_terms(hp.atom_of, hp.n_atom, hp.coords, hp.weights, hp.rho, g,
                                         hp.b, hp.C, hp.rho_x, gx)
            e0, _, _ = oracle.energy_potential(hp.coords, hp.weights, hp.rho, g, hp.b, hp.C)
            e, H = futs[k].result()
            chk.append({"rid": k, "n_grid": hp.n_grid, "energy_rel": abs(e - e0) / abs(e0),
                        "hess_max_abs": float(np.max(np.abs(H - H0)))})
        rec["vs_oracle"] = chk
    srv.close()
    return rec


def bench_served(args, torch, np, inputs, vv10):
    """The served stream alone as the JSON line's workload."""
    rec = served_stream(args, torch, np, inputs, vv10)
    out = {
        "metric": METRIC, "value": rec["throughput_pair_pert_per_s"], "unit": "pair*pert/s",
        "n_gpus": 1, "steps": rec["requests"], "warmup": rec["warmup"],
        "ms_per_step": rec["wall_s"] / rec["requests"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.prec], "data": "synthetic",
        "config": {"workload": "served", "precision": args.prec},
        "latency_s": rec["latency_s"], "served": rec, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water_20mer",
                    choices=["water_dimer", "water_hexamer", "water_20mer", "batch64", "served",
                             "trial_response", "gradient", "becke_hexamer", "becke_20mer"],
                    help="batch64: 64 random clusters of 1-30 waters, 1500 points/atom, "
                         "one graph launch per step")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the headline path (default: split-BF16 mixed)")
    ap.add_argument("--compare", default="fp64,fp32",
                    help="comma-separated precisions also timed on the same workload, each "
                         "compared element by element with the FP64 path ('none': no leg)")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served-stream leg of the single-molecule workloads")
    ap.add_argument("--no-oracle-rows", action="store_true",
                    help="skip the oracle checks on sampled rows")
    ap.add_argument("--shells", action="store_true",
                    help="store each atom's points in radial-shell order (same sample)")
    ap.add_argument("--screen", type=float, default=0.0,
                    help="contraction screening threshold tau (vv10_set_screening); with tau > 0 "
                         "the comparison leg is the same precision unscreened")
    ap.add_argument("--separate-energy", action="store_true",
                    help="energy and potential from vv10_energy_potential (own pair pass), "
                         "then vv10_hessian_terms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of 256 MiB first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this engine runs on one GPU; multi-GPU runs are not supported "
              "(--gpus 1 measures one GPU's throughput).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2208_14639_amd import inputs, vv10

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    vv10.load()
    prec = vv10.PRECISIONS[args.prec]

    if args.workload == "batch64":
        return bench_batch(args, torch, np, inputs, vv10)
    if args.workload == "served":
        return bench_served(args, torch, np, inputs, vv10)
    if args.workload == "trial_response":
        return bench_trial_response(args, torch, np, inputs, vv10)
    if args.workload == "gradient":
        return bench_gradient(args, torch, np, inputs, vv10)

    from paper_2208_14639_amd import autotune
    weighted = args.workload.startswith("becke_")
    if weighted:
        base = {"becke_hexamer": "water_hexamer", "becke_20mer": "water_20mer"}[args.workload]
        p = inputs.make_workload(base, weights="becke", radial_order=args.shells)
    else:
        p = inputs.make_workload(args.workload, radial_order=args.shells)
    compare = [c for c in args.compare.split(",") if c and c != "none" and c != args.prec]
    for c in compare:
        if c not in vv10.PRECISIONS:
            raise SystemExit(f"bench.py: unknown precision {c!r} in --compare")
    if args.screen > 0:
        compare = []                      # the comparison leg: the same precision unscreened
    n, na, P = p.n_grid, p.n_atom, p.n_pert
    tuned = {name: autotune.lookup(n, na, name) for name in ("fp64", "fp32", "bf16x3")}
    log(f"workload {args.workload}: N={n} atoms={na} P={P} prec={args.prec}")
    f64 = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
    coords, w, rho, grad = f64(p.coords), f64(p.weights), f64(p.rho), f64(p.grad_rho)
    atom_of = torch.as_tensor(p.atom_of, dtype=torch.int32).to(dev).contiguous()
    rho_x, grad_x = f64(p.rho_x), f64(p.grad_rho_x)
    w_x = f64(p.w_x) if weighted else None
    w_coef = torch.empty(n, dtype=torch.float64, device=dev) if weighted else None
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    f_rho = torch.empty(n, dtype=torch.float64, device=dev)
    f_gamma = torch.empty(n, dtype=torch.float64, device=dev)
    hess = torch.empty((P, P), dtype=torch.float64, device=dev)
    gradient = torch.empty(P, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    if args.copy_calibration:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    screen_stats = []

    def step(prec=prec, hess=hess, gradient=gradient, energy=energy, f_rho=f_rho, f_gamma=f_gamma,
             tau=args.screen, stages=None):
        h = vv10.vv10_prepare(p.b, p.C, n, na, coords, w, atom_of, rho, grad, prec, stream)
        try:
            tiles = tuned[vv10._prec_name(prec)]
            if tiles is not None:
                vv10.vv10_set_tiles(h, *tiles)
            if tau > 0:
                vv10.vv10_set_screening(h, tau)
            if stages is None:
                vv10.vv10_set_timing(h, True)
            else:
                vv10.vv10_set_timing_stages(h, stages)
            if args.separate_energy:
                vv10.vv10_energy_potential(h, energy, f_rho, f_gamma)
                if weighted:
                    vv10.vv10_nuclear_terms(h, P, rho_x, grad_x, hess=hess, grad=gradient,
                                            w_x=w_x, w_coef=w_coef)
                else:
                    vv10.vv10_hessian_terms(h, P, rho_x, grad_x, hess, gradient, None, None)
            else:
                vv10.vv10_nuclear_terms(h, P, rho_x, grad_x, hess=hess, grad=gradient, w_x=w_x,
                                        w_coef=w_coef, energy=energy, f_rho=f_rho, f_gamma=f_gamma)
            # each stage's latest run: the pair pass is the energy call's; read
            # once, where vv10_destroy would wait for the stream anyway
            st = vv10.vv10_stage_times(h)
            if tau > 0:
                screen_stats.append(vv10.vv10_screening_stats(h))
        finally:
            vv10.vv10_destroy(h)
        return st

    def timed(tag, **kw):
        for k in range(args.warmup):
            step(**kw)
            log(f"{tag}: warmup {k + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        stages = []
        t0 = time.perf_counter()
        for k in range(args.steps):
            stages.append(step(**kw))
            log(f"{tag}: step {k + 1}/{args.steps} done")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) / args.steps, {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}

    # the timed steps bracket only the stages the roofline reads with events
    # (each timed stage adds two event records to the stream); the other
    # stages' times come from a few steps after the timed region
    roof_stages = ["contract", "weights"] if weighted else ["contract"]

    def measure(tag, **kw):
        dt, roof_ms = timed(tag, stages=roof_stages, **kw)
        ns = min(args.steps, 5)
        stage_ms = {}
        for k in range(ns):
            st = step(**kw)
            stage_ms = {kk: stage_ms.get(kk, 0.0) + v / ns for kk, v in st.items()}
        log(f"{tag}: stage breakdown done")
        for kk in roof_stages:
            stage_ms[kk] = roof_ms[kk]
        return dt, stage_ms

    dt, stage_ms = measure(args.prec)
    pair_pert = float(n) * n * P
    value = pair_pert / dt

    t_con = stage_ms["contract"] * 1e-3
    mfma_key = {"fp64": "mfma_f64", "fp32": "mfma_f32", "bf16x3": "mfma_bf16"}[args.prec]
    # split-BF16 with moving weights and at most four 16-column blocks: the
    # library runs the main and the weight contraction as one kernel (the
    # contraction stage), and the weight stage is the weight packing alone
    fused_w = weighted and args.prec == "bf16x3" and args.screen == 0 and (P + 15) // 16 <= 4
    flops_con = FLOPS_PER_PAIR_PERT + (FLOPS_PER_PAIR_PERT_W if fused_w else 0)
    achieved = flops_con * pair_pert / t_con / 1e12
    # the weighted workload runs the same main contraction launch on the same
    # grid, unless the two contractions are fused (no counter record for that)
    traffic = None if fused_w else measured_traffic("contract", base if weighted else args.workload,
                                                    args.prec)
    roofline = dict(bound="mfma", kernel="k_contract_bf16x3_w" if fused_w else f"k_contract_{args.prec}",
                    achieved=achieved, peak=PEAKS_TFLOPS[mfma_key], unit="TFLOP/s",
                    frac=achieved / PEAKS_TFLOPS[mfma_key], traffic=traffic)
    if fused_w:
        roofline["flops_per_pair_pert"] = flops_con
    rec = None if fused_w else counter_record("contract", base if weighted else args.workload,
                                              args.prec)
    if rec is not None and "valu_issue_busy" in rec:
        # what limits the kernel, from the committed counter summary of the same launch
        roofline["issue"] = {"valu_issue_busy": rec["valu_issue_busy"], "mfma_busy": rec["mfma_busy"],
                             "source": rec["profile"]}
    # the pair integrals come from the grid pass unless --separate-energy
    pair_ms = stage_ms["pair"] if stage_ms["pair"] > 0 else stage_ms["grid"]

    out = {
        "metric": "VV10 Hessian grid-pair\u00b7perturbation/s, mixed vs FP64, at stated err; p99 latency",
        "value": value,
        "unit": "pair*pert/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f32+f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "n_grid": n, "n_atom": na, "n_pert": P,
                   "precision": args.prec, "compared": compare, "b": p.b, "C": p.C,
                   "seed": p.seed, "tiles": tuned[args.prec] or "automatic"},
        "roofline": roofline,
        "stage_ms": stage_ms,
        "pair_pass": {"kernel": "k_pair" if stage_ms["pair"] > 0 else "k_grid (fused)",
                      "pairs_per_s": float(n) * n / (pair_ms * 1e-3),
                      "roofline": pair_pass_roofline(p, "k_pair" if stage_ms["pair"] > 0 else "k_grid",
                                                     pair_ms, args.prec)},
        "step_calls": "vv10_energy_potential + vv10_hessian_terms" if args.separate_energy
                      else "vv10_nuclear_terms (energy, potential, Hessian, gradient)",
        "footprint_bytes": vv10.vv10_footprint_bytes(n, na, prec),
    }
    if not args.separate_energy:
        # the energy call on its own (its own pair pass, k_pair), timed apart
        # from the steps: a few untimed-step calls, the pass from HIP events
        e_ms = []
        e3, fr3, fg3 = torch.empty_like(energy), torch.empty_like(f_rho), torch.empty_like(f_gamma)
        for k in range(max(3, min(args.steps, 10))):
            h = vv10.vv10_prepare(p.b, p.C, n, na, coords, w, atom_of, rho, grad, prec, stream)
            try:
                vv10.vv10_set_timing(h, True)
                vv10.vv10_energy_potential(h, e3, fr3, fg3)
                e_ms.append(vv10.vv10_stage_times(h)["pair"])
            finally:
                vv10.vv10_destroy(h)
        e_ms = float(np.median(e_ms[1:]))
        out["energy_call"] = {"kernel": "k_pair", "pair_pass_ms": e_ms,
                              "pairs_per_s": float(n) * n / (e_ms * 1e-3),
                              "roofline": pair_pass_roofline(p, "k_pair", e_ms, args.prec)}
    if weighted:
        out["config"]["weights"] = "becke"
        if fused_w:
            # the weight rows are contracted inside `roofline`'s kernel
            out["weights_kernel"] = dict(fused_with="k_contract_bf16x3_w",
                                         packing_ms=stage_ms["weights"])
        else:
            t_w = stage_ms["weights"] * 1e-3
            aw = FLOPS_PER_PAIR_PERT_W * pair_pert / t_w / 1e12
            out["weights_kernel"] = dict(bound="mfma", kernel=f"k_wcontract_{args.prec}",
                                         achieved=aw, peak=PEAKS_TFLOPS[mfma_key],
                                         unit="TFLOP/s", frac=aw / PEAKS_TFLOPS[mfma_key],
                                         stage_ms=stage_ms["weights"])

    if args.shells:
        out["config"]["point_order"] = "radial shells"
    if args.screen > 0:
        act, tot = screen_stats[-1]
        out["config"]["screening_tau"] = args.screen
        out["screening"] = {"active_blocks": act, "total_blocks": tot,
                            "computed_fraction": act / tot,
                            "computed_pair_pert_per_s": value * act / tot,
                            "note": "value counts every pair; the contraction computed "
                                    "computed_fraction of its (16-point, 16-column) blocks"}
        hs = hess.clone()

    def outputs(hh, gg, ee, fr, fg):
        return dict(hess=hh.cpu().numpy(), grad=gg.cpu().numpy(), energy=ee.item(),
                    f_rho=fr.cpu().numpy(), f_gamma=fg.cpu().numpy())

    def resp_rows(pr):
        """Response rows of one untimed call (the inner sums of E_{G,G}), for
        the element-by-element and oracle-row comparisons."""
        h = vv10.vv10_prepare(p.b, p.C, n, na, coords, w, atom_of, rho, grad, vv10.PRECISIONS[pr], stream)
        try:
            tiles = tuned[pr]
            if tiles is not None:
                vv10.vv10_set_tiles(h, *tiles)
            rr = torch.empty((P, n), dtype=torch.float64, device=dev)
            rg = torch.empty_like(rr)
            vv10.vv10_nuclear_terms(h, P, rho_x, grad_x, resp_rho=rr, resp_gamma=rg, w_x=w_x)
            torch.cuda.synchronize()
            return rr.cpu().numpy(), rg.cpu().numpy()
        finally:
            vv10.vv10_destroy(h)

    results = {args.prec: outputs(hess, gradient, energy, f_rho, f_gamma)}
    if args.screen > 0:
        h2 = torch.empty_like(hess)
        g2 = torch.empty_like(gradient)
        e2 = torch.empty_like(energy)
        fr2, fg2 = torch.empty_like(f_rho), torch.empty_like(f_gamma)
        dt2, st2 = measure("unscreened", hess=h2, gradient=g2, energy=e2, f_rho=fr2, f_gamma=fg2,
                           tau=0.0)
        Hu = h2.cpu().numpy()
        out["vs_unscreened"] = {"ms_per_step": dt2 * 1e3, "value": pair_pert / dt2,
                                "speedup": dt2 / dt, "contract_ms": st2["contract"],
                                "screened_contract_ms": stage_ms["contract"],
                                "hess_change_normwise": float(np.max(np.abs(hs.cpu().numpy() - Hu))
                                                              / np.max(np.abs(Hu)))}
    for c in compare:
        h2 = torch.empty_like(hess)
        g2 = torch.empty_like(gradient)
        e2 = torch.empty_like(energy)
        fr2, fg2 = torch.empty_like(f_rho), torch.empty_like(f_gamma)
        dt2, st2 = measure(c, prec=vv10.PRECISIONS[c], hess=h2, gradient=g2, energy=e2,
                           f_rho=fr2, f_gamma=fg2)
        results[c] = outputs(h2, g2, e2, fr2, fg2)
        out[f"vs_{c}"] = {"precision": c, "ms_per_step": dt2 * 1e3, "value": pair_pert / dt2,
                          "speedup": dt2 / dt, "contract_ms": st2["contract"], "stage_ms": st2}

    # response rows of every path (one untimed call each)
    if not weighted:
        for pr in results:
            results[pr]["resp_rho"], results[pr]["resp_gamma"] = resp_rows(pr)
        log("response rows of every path done")

    # every mixed output against the FP64 GPU path, element by element
    if "fp64" in results:
        ref64 = results["fp64"]
        for pr, r in results.items():
            if pr == "fp64":
                continue
            e = errors_vs(r, ref64)
            e["within_stated_bounds"] = bool(
                e["energy_rel"] <= 1e-6 and e["hess_max_abs"] <= 1e-5
                and e["f_rho_normwise"] <= 1e-5 and e["f_gamma_normwise"] <= 1e-5
                and e["grad_normwise"] <= 1e-5)
            if pr == args.prec:
                out["errors_vs_fp64"] = e
            else:
                out[f"vs_{pr}"]["errors_vs_fp64"] = e

    # results of the last step: properties that hold at any size
    H = results[args.prec]["hess"]
    out["checks"] = {"hess_symmetric": bool(np.array_equal(H, H.T)),
                     "hess_row_sum_rel": float(np.max(np.abs(H.reshape(P, na, 3).sum(axis=1)))
                                               / np.max(np.abs(H)))}
    if not args.no_oracle_rows and not weighted:
        log("oracle rows (three places) running ...")
        out["errors_vs_oracle_rows"] = oracle_row_checks(p, results)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) running ...")
        cb, ref = cpu_baseline(p)
        out["cpu_baseline"] = cb
        if ref is not None:
            def errs(r):
                return {
                    "energy_rel": abs(r["energy"] - ref["E"]) / abs(ref["E"]),
                    "f_rho_normwise": float(np.max(np.abs(r["f_rho"] - ref["f_rho"])) / np.max(np.abs(ref["f_rho"]))),
                    "f_gamma_normwise": float(np.max(np.abs(r["f_gamma"] - ref["f_gamma"])) / np.max(np.abs(ref["f_gamma"]))),
                    "hess_normwise": float(np.max(np.abs(r["hess"] - ref["H"])) / np.max(np.abs(ref["H"]))),
                    "hess_max_abs": float(np.max(np.abs(r["hess"] - ref["H"]))),
                }
            out["errors_vs_oracle"] = errs(results[args.prec])
            for c in compare:
                out[f"vs_{c}"]["errors_vs_oracle"] = errs(results[c])
    else:
        out["cpu_baseline"] = None
    if not args.no_served and args.screen == 0 and not weighted:
        log("served stream running ...")
        rec = served_stream(args, torch, np, inputs, vv10)
        out["latency_s"] = rec["latency_s"]
        out["served"] = rec
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
