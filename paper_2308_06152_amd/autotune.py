"""Autotuner for the launch-level settings of a workload.

The kernels' tile shapes are fixed by their LDS and register layouts, and the
Krylov grids are sized from occupancy queries, so the settings left to pick per
workload are:
  vc_tail         the node limit below which the V-cycle's upward passes run
                  fused in one launch (0 = one launch per level);
  graphs          replay each coarse-GMRES step from a captured HIP graph;
  coarse_restart  the restart length of the inner coarse GMRES (it changes the
                  iteration counts, not the result's accuracy: every candidate
                  solves to the same tolerance).
Each candidate is timed on the workload itself (median of `reps` whole solves
after one warm-up) and the fastest kept.  Results are cached in a JSON file
keyed by the device architecture, the precision, the grid, the number of
right-hand sides and the method options, so a workload is tuned once per
machine type.
"""
from __future__ import annotations

import itertools
import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

VC_TAIL = (0, 70000, 300000, 1100000)
GRAPHS = (0, 1)
COARSE_RESTART = (8, 10, 12, 15, 20, 30)


def arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def key(nx, ny, bc, coarse_op, precision, nrhs, kvar) -> str:
    return (f"{arch()}|prec{precision}|{nx}x{ny}|bc{bc}|op{coarse_op}|nrhs{nrhs}"
            f"|{'vark' if kvar else 'constk'}")


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(grid, nrhs, opts, kvar, cache_path: str = DEFAULT_CACHE) -> dict:
    """The cached choice for this workload on this device type, or {}."""
    nx, ny, hx, hy, bc = grid
    kk = key(nx, ny, bc, opts.get("coarse_op", 0), opts.get("precision", 0), nrhs, kvar)
    e = load_cache(cache_path).get(kk)
    return dict(e["best"]) if e else {}


def _time_solves(H, torch, grid, k, kconst, b, opts, reps):
    nx, ny, hx, hy, bc = grid
    S = H.Solver(nx, ny, hx, hy, bc, k=k, kconst=kconst, **opts)
    try:
        x = torch.zeros_like(b)
        S.solve(b, x)  # warm-up (graph capture, first-use allocations)
        ts, info = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = S.solve(b, x)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        if not all(i["converged"] for i in info):
            return float("inf"), info
        return sorted(ts)[len(ts) // 2], info
    finally:
        S.close()


def tune(grid, b, opts, k=None, kconst=0.0, reps=3, cache_path: str = DEFAULT_CACHE,
         retune: bool = False, log=print, vc_tail=VC_TAIL, graphs=GRAPHS,
         coarse_restart=COARSE_RESTART) -> dict:
    """Pick vc_tail, graphs and coarse_restart for solving b (device tensor,
    one or more right-hand sides) on `grid` = (nx, ny, hx, hy, bc) with the
    method options `opts`.  Returns the chosen settings (merged into opts by
    the caller); the choice and every candidate's time go to the cache."""
    import torch
    from . import helmdefl as H
    nx, ny, hx, hy, bc = grid
    nrhs = 1 if b.dim() == 2 else int(b.shape[0])
    kk = key(nx, ny, bc, opts.get("coarse_op", 0), opts.get("precision", 0), nrhs,
             k is not None)
    cache = load_cache(cache_path)
    if kk in cache and not retune:
        return dict(cache[kk]["best"])
    trials = []
    # graphs replay only the single-right-hand-side coarse steps
    graphs = graphs if nrhs == 1 else (0,)
    for vt, gr, cr in itertools.product(vc_tail, graphs, coarse_restart):
        o = dict(opts, vc_tail=vt, graphs=gr, coarse_restart=cr)
        t, info = _time_solves(H, torch, grid, k, kconst, b, o, reps)
        trials.append({"vc_tail": vt, "graphs": gr, "coarse_restart": cr, "seconds": t,
                       "outer_iters": max(i["outer_iters"] for i in info),
                       "inner_iters": sum(i["inner_iters_total"] for i in info)})
        log(f"autotune {kk}: vc_tail={vt} graphs={gr} coarse_restart={cr}: {t * 1e3:.1f} ms")
    best = min(trials, key=lambda r: r["seconds"])
    choice = {n: best[n] for n in ("vc_tail", "graphs", "coarse_restart")}
    cache = load_cache(cache_path)
    cache[kk] = {"best": choice, "trials": trials,
                 "opts": {n: v for n, v in opts.items() if isinstance(v, (int, float))}}
    save_cache(cache, cache_path)
    return choice
