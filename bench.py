#!/usr/bin/env python3
"""Benchmark of the VV10 Hessian-term engine on one MI355X.

One step is one pass of the whole hot path over one synthetic molecule
already resident in HBM: vv10_prepare (per-point prep) -> vv10_nuclear_terms
with the energy, potential, Hessian-term and gradient outputs (one pass over
the pairs for the pair integrals E..C and the grid-position terms, the
potential and energy, perturbation packing, MFMA contraction, assembly) ->
vv10_destroy.  --separate-energy times vv10_energy_potential (its own pair
pass) followed by vv10_hessian_terms instead.

Metric: grid-pair x perturbation per second, N^2 P / t_step, with N^2 the
ordered pairs (self pairs included) and P = 3 N_atom.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (the perturbation contraction, timed with HIP events recorded by the
library on the plan's stream), the pair pass against the vector peak (the
step's fused grid pass, and the energy call's own pair kernel timed apart
from the steps) and a CPU baseline (the FP64 oracle on the host, rank 0
only).
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(rels):
    h = hashlib.sha256()
    for rel in rels:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
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


def cpu_baseline(p, budget_s=30.0):
    """FP64 oracle on the host.  Full workload when it fits the budget, else
    the dominant O(N^2 P) step (response rows, and with weight derivatives the
    weight integrals of the same rows) on a row sample."""
    import oracle
    g, gx = oracle.problem_inputs(p)
    n, P = p.n_grid, p.n_pert
    est_rate = 3e9 * oracle.num_threads() / 8      # pair*pert/s, measured order of magnitude
    if p.w_x is not None:
        def rows(k):
            oracle.response_rows(0, k, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
            oracle.weight_integrals(p.coords, p.rho, g, p.b, p.C, p.w_x, 0, k)
        k, dt, _ = row_sample(rows, n)
        return dict(value=k * n * P / dt, unit="pair*pert/s", cores=oracle.num_threads(),
                    kind="oracle", seconds=dt,
                    sample=f"response rows and weight integrals of rows 0..{k} of N={n}, P={P} "
                           f"(dominant N^2 P steps incl. one full pair-integral pass)"), None
    if n * n * P / est_rate <= budget_s:
        t0 = time.perf_counter()
        H, _ = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                    p.rho_x, gx)
        e0, fr0, fg0 = oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)
        dt = time.perf_counter() - t0
        return dict(value=n * n * P / dt, unit="pair*pert/s", cores=oracle.num_threads(),
                    kind="oracle", seconds=dt,
                    sample=f"whole workload: energy, potential and Hessian terms, N={n}, P={P}"), \
            dict(H=H, E=e0, f_rho=fr0, f_gamma=fg0)
    k, dt, _ = row_sample(
        lambda k: oracle.response_rows(0, k, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx), n)
    return dict(value=k * n * P / dt, unit="pair*pert/s", cores=oracle.num_threads(),
                kind="oracle", seconds=dt,
                sample=f"response rows 0..{k} of N={n}, P={P} (dominant N^2 P step incl. one "
                       f"full pair-integral pass)"), None


def bench_batch(args, torch, np, inputs, vv10):
    """64 molecules of uneven size in one graph launch per step."""
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
        "metric": "VV10 Hessian grid-pair\u00b7perturbation/s, mixed vs FP64, at stated err; p99 latency",
        "value": pair_pert / dt, "unit": "pair*pert/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f32+f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "batch64", "n_mol": len(probs), "waters": sizes, "n_pa": 1500,
                   "precision": args.prec, "work_items": n_items, "persistent_workgroups": n_wg},
        "roofline": None, "cpu_baseline": None,
    }
    # CPU baseline: the whole oracle on the three smallest molecules, whose
    # results also check the batch's
    if not args.no_cpu_baseline:
        import oracle
        order = np.argsort([p.n_grid for p in probs])[:3]
        errs = []
        work, secs = 0.0, 0.0
        for m in order:
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
        out["cpu_baseline"] = dict(value=work / secs, unit="pair*pert/s", cores=oracle.num_threads(),
                                   kind="oracle", seconds=secs,
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


def bench_served(args, torch, np, inputs, vv10, pool_size=16, n_requests=96, n_warm=8):
    """Poisson stream of requests (1-30 waters, 1000-2500 points/atom) through
    the continuous-batching server; p50/p99 latency and throughput."""
    from paper_2208_14639_amd.serve import GpuExecutor, Request, Server
    rng = np.random.default_rng(1005)
    pool = []
    for k in range(pool_size):
        pool.append(inputs.make_problem(int(rng.integers(1, 31)), int(rng.integers(1000, 2501)),
                                        3000 + k))
        log(f"generated {k + 1}/{pool_size} molecules (N={pool[-1].n_grid})")
    # single-slot service times (also the results alone)
    alone, service = [], []
    for k, p in enumerate(pool):
        with vv10.Plan(p, prec=args.prec, tiles="auto") as pl:
            pl.hessian_terms(p.rho_x, p.grad_rho_x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, _, _ = pl.energy_potential()
            H = pl.hessian_terms(p.rho_x, p.grad_rho_x)["hess"]
            torch.cuda.synchronize()
            service.append(time.perf_counter() - t0)
            alone.append((e.item(), H.cpu().numpy()))
        log(f"alone {k + 1}/{pool_size}: {service[-1] * 1e3:.1f} ms")
    rate = 0.7 / float(np.mean(service))             # 70% of the single-slot capacity
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = rng.integers(0, pool_size, size=n_requests)
    ex = GpuExecutor(prec=args.prec, n_slots=4)
    budget = 96 * 1024 ** 3
    srv = Server(ex, budget, n_slots=4)
    futs = [srv.submit(Request(k, f"m{m}", pool[m]), at=float(t))
            for k, (m, t) in enumerate(zip(which, arrivals))]
    t0 = time.perf_counter()
    srv.run_until_idle(timeout_s=240)
    wall = time.perf_counter() - t0
    max_diff, same = 0.0, True
    for k, m in enumerate(which):
        e, H = futs[k].result()
        same &= bool(np.array_equal(H, alone[m][1])) and e == alone[m][0]
        max_diff = max(max_diff, float(np.max(np.abs(H - alone[m][1]))))
    st = srv.stats(skip=n_warm)
    srv.close()
    out = {
        "metric": "VV10 Hessian grid-pair\u00b7perturbation/s, mixed vs FP64, at stated err; p99 latency",
        "value": st["throughput_pair_pert_per_s"], "unit": "pair*pert/s", "n_gpus": 1,
        "steps": n_requests, "warmup": n_warm, "ms_per_step": wall / n_requests * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f32+f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "served", "pool": pool_size, "requests": n_requests,
                   "arrival_rate_per_s": rate, "rate_fraction_of_single_slot": 0.7,
                   "slots": 4, "budget_bytes": budget, "precision": args.prec},
        "latency_s": {"p50": st["p50_s"], "p99": st["p99_s"], "mean": st["mean_s"]},
        "single_slot_mean_s": float(np.mean(service)),
        "served": st,
        "results_identical_alone_and_in_mix": same, "max_abs_diff_vs_alone": max_diff,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water_hexamer",
                    choices=["water_dimer", "water_hexamer", "water_20mer", "batch64", "served",
                             "trial_response", "gradient", "becke_hexamer", "becke_20mer"],
                    help="batch64: 64 random clusters of 1-30 waters, 1500 points/atom, "
                         "one graph launch per step")
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the headline path (default: split-BF16 mixed)")
    ap.add_argument("--compare", default="fp64", choices=["fp64", "fp32", "bf16x3", "none"],
                    help="also time this precision on the same workload (the 'vs FP64' ratio)")
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
    if args.screen > 0:
        args.compare = args.prec          # the comparison leg: unscreened
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
    achieved = FLOPS_PER_PAIR_PERT * pair_pert / t_con / 1e12
    # the weighted workload runs the same main contraction launch on the same grid
    traffic = measured_traffic("contract", base if weighted else args.workload, args.prec)
    roofline = dict(bound="mfma", kernel=f"k_contract_{args.prec}", achieved=achieved,
                    peak=PEAKS_TFLOPS[mfma_key], unit="TFLOP/s",
                    frac=achieved / PEAKS_TFLOPS[mfma_key], traffic=traffic)
    rec = counter_record("contract", base if weighted else args.workload, args.prec)
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
                   "precision": args.prec, "b": p.b, "C": p.C, "seed": p.seed,
                   "tiles": tuned[args.prec] or "automatic"},
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
        t_w = stage_ms["weights"] * 1e-3
        aw = FLOPS_PER_PAIR_PERT_W * pair_pert / t_w / 1e12
        out["config"]["weights"] = "becke"
        out["weights_kernel"] = dict(bound="mfma", kernel=f"k_wcontract_{args.prec}", achieved=aw,
                                     peak=PEAKS_TFLOPS[mfma_key], unit="TFLOP/s",
                                     frac=aw / PEAKS_TFLOPS[mfma_key], stage_ms=stage_ms["weights"])

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
    cmp = None
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
    elif args.compare != "none" and args.compare != args.prec:
        h2 = torch.empty_like(hess)
        g2 = torch.empty_like(gradient)
        e2 = torch.empty_like(energy)
        fr2, fg2 = torch.empty_like(f_rho), torch.empty_like(f_gamma)
        dt2, st2 = measure(args.compare, prec=vv10.PRECISIONS[args.compare], hess=h2, gradient=g2,
                           energy=e2, f_rho=fr2, f_gamma=fg2)
        cmp = dict(precision=args.compare, ms_per_step=dt2 * 1e3, value=pair_pert / dt2,
                   stage_ms=st2, hess=h2.cpu().numpy(), energy=e2.item(),
                   f_rho=fr2.cpu().numpy(), f_gamma=fg2.cpu().numpy())
        out[f"vs_{args.compare}"] = {"precision": args.compare, "ms_per_step": dt2 * 1e3,
                                     "value": pair_pert / dt2, "speedup": dt2 / dt,
                                     "contract_ms": st2["contract"], "stage_ms": st2}

    # results of the last step, checked against the oracle when it ran in full
    H = hess.cpu().numpy()
    out["checks"] = {"hess_symmetric": bool(np.array_equal(H, H.T)),
                     "hess_row_sum_rel": float(np.max(np.abs(H.reshape(P, na, 3).sum(axis=1)))
                                               / np.max(np.abs(H)))}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) running ...")
        cb, ref = cpu_baseline(p)
        out["cpu_baseline"] = cb
        if ref is not None:
            def errs(e, fr, fg, HH):
                return {
                    "energy_rel": abs(e - ref["E"]) / abs(ref["E"]),
                    "f_rho_normwise": float(np.max(np.abs(fr - ref["f_rho"])) / np.max(np.abs(ref["f_rho"]))),
                    "f_gamma_normwise": float(np.max(np.abs(fg - ref["f_gamma"])) / np.max(np.abs(ref["f_gamma"]))),
                    "hess_normwise": float(np.max(np.abs(HH - ref["H"])) / np.max(np.abs(ref["H"]))),
                    "hess_max_abs": float(np.max(np.abs(HH - ref["H"]))),
                }
            out["errors_vs_oracle"] = errs(energy.item(), f_rho.cpu().numpy(), f_gamma.cpu().numpy(), H)
            if cmp is not None:
                out[f"vs_{args.compare}"]["errors_vs_oracle"] = errs(cmp["energy"], cmp["f_rho"],
                                                                      cmp["f_gamma"], cmp["hess"])
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
