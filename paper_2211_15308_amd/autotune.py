"""Autotuner of the launch schedule and tiling (batched and single-problem solves).

Launch parameters that trade work against launches are chosen by timing the caller's own
workload on the device:

  * mg_nu      -- red-black sweep pairs per level in the multigrid V-cycle (1 or 2): more
                  smoothing per V-cycle, fewer PCG iterations;
  * step_rtol  -- residual reduction of each FP32 multigrid-PCG run inside the FP64 iterative
                  refinement (1e-4, 1e-5, 1e-6): fewer, longer runs or more, shorter ones;
  * mid_tile   -- (batches) tile edge of the intermediate multigrid levels: 16 x 16 tiles spread a
                  latency-bound level over more workgroups, 32 x 32 tiles re-read less halo; 0
                  chooses per level by tile count.  Searched after (mg_nu, step_rtol), at the best
                  of those.

Every candidate is run once untimed (it measures its launch schedule and captures its graphs),
then timed; the fastest wins.  Choices are cached as JSON keyed by the workload signature (the
sorted (n, log10 K, log10 mu) of the instances), the kind of solve, the arithmetic (mixed) and the
GPU architecture, so a repeated workload is not timed again.
"""
import hashlib
import json
import os
import time

CANDIDATES = [(nu, tau) for nu in (1, 2) for tau in (1e-4, 1e-5, 1e-6)]


def default_cache_path():
    base = os.environ.get("FDD_AUTOTUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2211_15308_amd", "autotune.json")


def signature(problems):
    import math
    items = sorted((p.n, round(math.log10(p.K), 2), round(math.log10(p.mu), 2)) for p in problems)
    return hashlib.sha256(json.dumps(items).encode()).hexdigest()[:16]


def arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _load(path):
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_batch(batch, bs, xs, base_opts=None, reps=2, cache_path=None, candidates=CANDIDATES,
               force=False, mid_tiles=(16, 32)):
    """Returns (opts, record) with the fastest (mg_nu, step_rtol) for this batch, and sets the
    batch's fastest intermediate-level tile edge (recorded as mid_tile and tile_edges).

    base_opts supplies every other option (tolerances, graph use).  The record holds the key,
    the per-candidate timings (ms per batch solve) and whether it came from the cache.
    """
    import torch

    from . import fdd as F
    opts = base_opts or F.opts_default()
    key = "|".join(["solve_batched", signature(batch.problems), "mixed", arch(),
                    f"rtol={opts.outer_rtol:g}", f"inner={opts.inner_rtol:g}", "tiles"])
    path = cache_path or default_cache_path()
    table = _load(path)
    if key in table and not force:
        rec = dict(table[key], cached=True)
        batch.set_mid_tile(rec["mid_tile"])
        return _with(F, opts, rec["mg_nu"], rec["step_rtol"]), rec

    def timed(o):
        batch.solve(bs, xs, o)  # measures the schedule, captures the graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.solve(bs, xs, o)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    timings = {}
    batch.set_mid_tile(0)
    for nu, tau in candidates:
        timings[f"nu={nu},tau={tau:g},mid=0"] = timed(_with(F, opts, nu, tau))
    best = min(candidates, key=lambda c: timings[f"nu={c[0]},tau={c[1]:g},mid=0"])
    best_mid, best_ms = 0, timings[f"nu={best[0]},tau={best[1]:g},mid=0"]
    for mid in mid_tiles:
        batch.set_mid_tile(mid)
        ms = timed(_with(F, opts, best[0], best[1]))
        timings[f"nu={best[0]},tau={best[1]:g},mid={mid}"] = ms
        if ms < best_ms:
            best_mid, best_ms = mid, ms
    batch.set_mid_tile(best_mid)
    rec = {"key": key, "mg_nu": best[0], "step_rtol": best[1], "mid_tile": best_mid,
           "tile_edges": batch.tile_edges(), "ms_per_batch": timings, "instances": batch.count}
    table[key] = rec
    _store(path, table)
    return _with(F, opts, best[0], best[1]), dict(rec, cached=False)


def _with(F, opts, nu, tau):
    o = F.FddOpts()
    for name, _ in F.FddOpts._fields_:
        setattr(o, name, getattr(opts, name))
    o.mg_nu = nu
    o.step_rtol = tau
    return o


def tune_solves(cases, base_opts=None, reps=1, cache_path=None, candidates=CANDIDATES, force=False):
    """The same choice for single-problem solves: cases = [(problem, P table, H table, b, x)], timed
    over one pass through all cases per candidate.  Returns (opts, record)."""
    import torch

    from . import fdd as F
    opts = base_opts or F.opts_default()
    key = "|".join(["solve", signature([c[0] for c in cases]), "mixed", arch(),
                    f"rtol={opts.outer_rtol:g}", f"inner={opts.inner_rtol:g}"])
    path = cache_path or default_cache_path()
    table = _load(path)
    if key in table and not force:
        rec = dict(table[key], cached=True)
        return _with(F, opts, rec["mg_nu"], rec["step_rtol"]), rec
    timings = {}
    for nu, tau in candidates:
        o = _with(F, opts, nu, tau)
        for P, TP, TH, b, x in cases:
            P.solve(TP, TH, b, x, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for P, TP, TH, b, x in cases:
                P.solve(TP, TH, b, x, o)
        torch.cuda.synchronize()
        timings[f"nu={nu},tau={tau:g}"] = 1e3 * (time.perf_counter() - t0) / (reps * len(cases))
    best = min(candidates, key=lambda c: timings[f"nu={c[0]},tau={c[1]:g}"])
    rec = {"key": key, "mg_nu": best[0], "step_rtol": best[1], "ms_per_solve": timings}
    table[key] = rec
    _store(path, table)
    return _with(F, opts, best[0], best[1]), dict(rec, cached=False)
