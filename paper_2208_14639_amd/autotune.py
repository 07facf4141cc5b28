"""Tile-shape autotuner for the VV10 library.

Two knobs decide how the O(N^2) work is cut into workgroups:
  * jsplit  -- j splits of the perturbation contraction (more splits fill
               the last round of workgroups better but add partial sums);
  * bgroups -- atom groups of the grid-term pass (more groups give more
               waves but more partial pair integrals).
For a problem size the tuner times candidate values of each knob with the
library's own per-stage HIP events (jsplit on the contraction plus the
assembly that sums its partials, bgroups on the grid pass; a fresh plan per
call, one untimed call and `repeats` timed ones), keeps the fastest, and
caches the choice in a
JSON file keyed by device architecture, precision and size bucket:
    "<arch>:<prec>:P<16-column blocks>:N<points, rounded up to 8192>"
Plans and batches take the cached tiles through vv10_set_tiles; sizes with
no entry use the library's automatic choice.

Command line (on a GPU):
    python -m paper_2208_14639_amd.autotune --workload water_hexamer --prec bf16x3
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
ARCH = "gfx950"


def bucket_key(n_grid: int, n_atom: int, prec: str) -> str:
    ncb = (3 * n_atom + 15) // 16
    nb = (n_grid + 8191) // 8192
    return f"{ARCH}:{prec}:P{ncb}:N{nb * 8192}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(n_grid: int, n_atom: int, prec: str, cache: dict | None = None):
    """(jsplit, bgroups) for this size, or None when the bucket is untuned."""
    cache = load_cache() if cache is None else cache
    rec = cache.get(bucket_key(n_grid, n_atom, prec))
    if not rec:
        return None
    return int(rec["jsplit"]), int(rec["bgroups"])


def candidates(auto: int, lo: int, hi: int):
    vals = {auto, max(lo, auto // 2), max(lo, (2 * auto) // 3), min(hi, (3 * auto) // 2),
            min(hi, 2 * auto), max(lo, auto - 1), min(hi, auto + 1)}
    return sorted(v for v in vals if lo <= v <= hi)


def _time_stages(problem, prec, tiles, stages, repeats, rx, gx):
    """Fastest summed time of `stages` over `repeats` calls, each on a fresh
    plan (so the grid pass forms the pair integrals, as on a new geometry),
    after one untimed call; only the scored stages carry timing events."""
    import torch
    from . import vv10
    ms, used = [], None
    for r in range(repeats + 1):
        with vv10.Plan(problem, prec=prec, tiles=tiles) as pl:
            vv10.vv10_set_timing_stages(pl.handle, stages)
            pl.nuclear_terms(rx, gx, hess=True, grad=True, energy=True, potential=True)
            st = vv10.vv10_stage_times(pl.handle)
            used = vv10.vv10_get_tiles(pl.handle)
            torch.cuda.synchronize()
        if r > 0:
            ms.append(sum(st[s] for s in stages))
    return min(ms), used


def tune(problem, prec: str = "bf16x3", repeats: int = 3, log=print) -> dict:
    """Tune one problem size; returns the record stored in the cache."""
    import torch
    from . import vv10
    dev = torch.device("cuda")
    rx = torch.as_tensor(problem.rho_x, dtype=torch.float64).to(dev).contiguous()
    gx = torch.as_tensor(problem.grad_rho_x, dtype=torch.float64).to(dev).contiguous()
    with vv10.Plan(problem, prec=prec) as pl:
        auto_j, auto_b = vv10.vv10_get_tiles(pl.handle)
    npad = ((problem.n_grid + 255) // 256) * 256
    # j splits: the contraction and the assembly, which sums the splits' partials
    best_j, best_jt = auto_j, None
    for j in candidates(auto_j, 1, max(1, npad // 256)):
        t, (jj, _) = _time_stages(problem, prec, (j, auto_b), ["contract", "assemble"], repeats, rx, gx)
        log(f"  jsplit {j} (effective {jj}): contract + assembly {t:.3f} ms")
        if best_jt is None or t < best_jt * 0.99:
            best_j, best_jt = jj, t
    best_b, best_bt = auto_b, None
    for bgr in candidates(auto_b, 1, problem.n_atom):
        t, (_, bb) = _time_stages(problem, prec, (best_j, bgr), ["grid"], repeats, rx, gx)
        log(f"  bgroups {bgr} (effective {bb}): grid {t:.3f} ms")
        if best_bt is None or t < best_bt * 0.99:
            best_b, best_bt = bb, t
    return {"jsplit": best_j, "bgroups": best_b, "contract_assemble_ms": best_jt, "grid_ms": best_bt,
            "auto": [auto_j, auto_b], "n_grid": problem.n_grid, "n_atom": problem.n_atom}


def main(argv=None):
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2208_14639_amd import inputs
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="water_hexamer", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args(argv)
    p = inputs.make_workload(args.workload)
    print(f"tuning {args.workload} ({p.n_grid} points, {p.n_pert} perturbations) {args.prec}", flush=True)
    rec = tune(p, args.prec, args.repeats, log=lambda *a: print(*a, flush=True))
    cache = load_cache(args.cache)
    cache[bucket_key(p.n_grid, p.n_atom, args.prec)] = rec
    save_cache(cache, args.cache)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
