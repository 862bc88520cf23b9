#!/usr/bin/env python3
"""Benchmark: Helmholtz solves/s to a 1e-6 relative residual on one MI355X.

One step = one complete solve of the large plain-method workload: the unit
square, 4097 x 4097 nodes, constant k = 800, first-order Sommerfeld boundary,
Gaussian source (sigma = 2h) at the centre, complex128, APD preconditioner
(Bezier deflation vectors, ReD-Glk2 coarse operator, coarse GMRES(15) to 0.1,
one CSLP V-cycle), FGMRES(50) to 1e-6.  Inputs are resident on the GPU before
the timed region.

Prints ONE JSON line with the contract fields plus:
  roofline      the dominant kernel's algorithmic HBM bytes / its average
                launch time, against the 8 TB/s HBM peak.  The solves are
                timed twice: `value` from a region with no kernel timing, then
                the same number of solves with HIP events recorded on the
                solver's stream around each launch of that kernel (their
                wall time is `ms_per_step_with_events`);
  cpu_baseline  the CPU oracle (OpenMP build, all host threads; a one-thread
                figure beside it) on the same workload: whole solves timed
                on small grids; on large ones a bounded sample,
                extrapolated to solves/s with the GPU run's iteration
                counts.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Helmholtz solves/s to 1e-6 rel. residual; stencil+V-cycle HBM GB/s vs peak"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "small", "wedge", "layered", "adjoint"],
                    default="large",
                    help="large: 4097^2 k=800 Sommerfeld (the headline); small: 129^2 "
                         "Dirichlet k=20; wedge: the 1153 x 1921 three-layer model at 40 Hz; "
                         "layered: 2049 x 1025 layered model, --nrhs sources at --freq; "
                         "adjoint: misfit gradients on 1025 x 513 with 16 shots at 10 Hz")
    ap.add_argument("--nrhs", type=int, default=64, help="layered: sources solved together")
    ap.add_argument("--freq", type=float, default=10.0, help="layered: frequency in Hz")
    ap.add_argument("--freqs", default="",
                    help="layered: comma-separated frequencies (Hz); one step solves the "
                         "--nrhs sources at each of them, one batched solve (and one handle) per "
                         "frequency")
    ap.add_argument("--batch", type=int, choices=[0, 1], default=1,
                    help="layered: 1 = one batched solve of all sources, 0 = one after another")
    ap.add_argument("--graphs", type=int, choices=[0, 1], default=0,
                    help="1 = coarse-GMRES steps replayed from captured HIP graphs")
    ap.add_argument("--vc-tail", type=int, default=300000,
                    help="FP64 V-cycle: largest level (nodes) whose upward pass and those of "
                         "the levels below run fused in one launch (0 = one launch per level)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed_c64basis"], default="fp64",
                    help="mixed: complex64 fine-grid CSLP V-cycle and smoother inside the FP64 "
                         "solve (coarse solve FP64); mixed_c64basis: also the coarse-GMRES "
                         "basis in complex64")
    ap.add_argument("--roofline-kernel", default="mupdate",
                    help="kernel class whose roofline is reported (default: the Gram-Schmidt "
                         "update, the kernel with the largest share of the solve's kernel time)")
    ap.add_argument("--roofline-level", type=int, default=1,
                    help="multigrid level of the timed kernel (-1 = any)")
    ap.add_argument("--autotune", choices=["off", "cache", "run"], default="cache",
                    help="cache: take vc_tail / graphs / coarse restart from the autotuner's "
                         "cache when it holds this workload on this device type (else the "
                         "defaults); run: time the candidates first and record the choice; "
                         "off: the defaults")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: the package's autotune_cache.json)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (out = in * 1) three times, "
                         "the reference for scaling rocprofv3 byte counters")
    return ap.parse_args()


def kernels_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "hd_common.h"):
        with open(os.path.join(ROOT, "paper_2308_06152_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, coarse_restart):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if
    absent, taken on a different version of the kernels or with another coarse
    restart (which sets the average number of basis vectors per launch)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(f"{kernel}@{workload}")
    if not e or e.get("kernels_sha") != kernels_hash():
        return None
    if e.get("coarse_restart", coarse_restart) != coarse_restart:
        return None
    return e.get("bytes_per_launch")


def host_cpu():
    """The host CPU's model name and the threads this process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def _oracle_problem(oracle, w, coarsest_nodes, **kw):
    kw.setdefault("coarse_restart", w.coarse_restart)
    return oracle.Problem(w.nx, w.ny, w.hx, w.hy, bc=w.bc, k=w.kfield(), kconst=w.kconst,
                          coarse_op=w.coarse_op, coarsest_nodes=coarsest_nodes, **kw)


def cpu_baseline_full(w, coarsest_nodes, coarse_restart, reps=5):
    """Time whole oracle solves of the workload (small grids), with the coarse
    restart of the GPU run: the median of `reps` solves with all host threads,
    and of 3 with one thread."""
    import oracle
    oracle.build(force=False)
    P = _oracle_problem(oracle, w, coarsest_nodes, coarse_mode=oracle.CMODE_TOL,
                        coarse_tol=w.coarse_tol, coarse_iters=w.coarse_maxit,
                        coarse_restart=coarse_restart)
    b = w.rhs()
    model, nthr = host_cpu()
    res = {}
    for th, n in ((nthr, reps), (1, 3)):
        oracle.set_threads(th)
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            _, inf = oracle.fgmres(P, b, restart=w.restart, tol=w.tol, maxit=500)
            ts.append(time.perf_counter() - t0)
        res[th] = (sorted(ts)[len(ts) // 2], inf)
    oracle.set_threads(nthr)
    t, inf = res[nthr]
    return {
        "value": 1.0 / t, "unit": "solves/s", "cores": nthr, "kind": "oracle",
        "sample": (f"whole oracle solves of the same workload ({w.nx}x{w.ny}): median of {reps} "
                   f"with {nthr} threads {t:.3f} s, median of 3 with 1 thread "
                   f"{res[1][0]:.3f} s; {inf.iters} outer / {inf.inner_total} inner iterations, "
                   f"relres {inf.relres:.2e}; host {model}"),
        "value_1thread": 1.0 / res[1][0],
        "host": model,
    }


def cpu_baseline(w, info, coarsest_nodes, coarse_restart):
    """Time the oracle on a bounded sample of the workload and extrapolate.

    Sample (C oracle, full grid, coarse restart m of the GPU run, with all host
    threads and again with one): one A_h apply; one coarse GMRES solve of m and
    one of 2m fixed iterations, whose difference C is one whole inner cycle
    (m steps, the cycle's solution update and the restart residual); one
    A-DEF1 application with an m-iteration coarse solve (the fine-grid part of
    an outer iteration plus one cycle).  Estimate of one solve =
    outer * (A_h + A-DEF1 - C) + (inner_total / m) * C, with the GPU run's
    counts; the outer Gram-Schmidt on the fine grid is left out (it favours
    the CPU)."""
    import oracle
    from paper_2308_06152_amd import inputs
    oracle.build(force=False)
    m = coarse_restart
    P = _oracle_problem(oracle, w, coarsest_nodes, coarse_mode=oracle.CMODE_FIXED,
                        coarse_iters=m, coarse_restart=m)
    nxc, nyc = oracle.coarse_dims(P)
    v = inputs.random_complex((w.ny, w.nx), 11)
    v1 = inputs.random_complex((nyc, nxc), 12)
    model, nthr = host_cpu()

    def timed(f, *args):
        t0 = time.perf_counter()
        f(*args)
        return time.perf_counter() - t0

    def sample():
        oracle.helm_apply(P, v)  # warm-up: thread start, first touch of the output
        t_a = timed(oracle.helm_apply, P, v)
        t_m = timed(oracle.coarse_solve, P, v1)
        t_2m = timed(oracle.coarse_solve, P.replace(coarse_iters=2 * m), v1)
        t_d = timed(oracle.deflate_apply, P, v, oracle.DEFL_ADEF1)
        cycle = max(t_2m - t_m, 0.0)
        est = (info["outer_iters"] * max(t_a + t_d - cycle, 0.0)
               + info["inner_iters_total"] / m * cycle)
        return est, (t_a, t_m, t_2m, t_d)

    res = {}
    for th in (nthr, 1):
        oracle.set_threads(th)
        res[th] = sample()
    oracle.set_threads(nthr)
    est, (t_a, t_m, t_2m, t_d) = res[nthr]
    return {
        "value": 1.0 / est, "unit": "solves/s", "cores": nthr, "kind": "oracle",
        "sample": (f"C oracle with {nthr} threads on the full {w.nx}x{w.ny} grid, coarse "
                   f"restart {m}: A_h apply {t_a:.2f}s, coarse GMRES {m} it {t_m:.2f}s / "
                   f"{2 * m} it {t_2m:.2f}s, A-DEF1 with {m} inner it {t_d:.2f}s (sample "
                   f"{sum(res[nthr][1]):.1f}s); extrapolated to {info['outer_iters']} outer + "
                   f"{info['inner_iters_total']} inner iterations = {est:.0f}s per solve; the "
                   f"same sample with 1 thread ({sum(res[1][1]):.1f}s) gives {res[1][0]:.0f}s "
                   f"per solve; host {model}"),
        "est_seconds_per_solve": est,
        "value_1thread": 1.0 / res[1][0],
        "host": model,
    }


def adjoint_bench(a, torch, H, inputs):
    """Misfit gradients per second: one step = one forward (batched over the
    shots) + adjoint solve + gradient accumulation, J(s) and dJ/ds."""
    from paper_2308_06152_amd import adjoint
    c = inputs.adjoint_case()
    omega = 2 * 3.141592653589793 * c["freq"]
    grid = (c["nx"], c["ny"], c["h"], c["h"], H.BC_SOMMERFELD)
    opts = dict(coarse_op=H.COARSE_REDGLK2, coarse_mode=H.CMODE_TOL, coarse_tol=0.1,
                coarse_iters=300, coarse_restart=15, restart=20, tol=1e-6, batch=a.batch,
                graphs=a.graphs, vc_tail=a.vc_tail)
    src = torch.from_numpy(c["sources"]).cuda()
    rec = torch.from_numpy(c["rec"]).cuda()
    kt = (omega * torch.sqrt(torch.from_numpy(c["s_true"]))).cuda()
    St = H.Solver(c["nx"], c["ny"], c["h"], c["h"], H.BC_SOMMERFELD, k=kt, **opts)
    ut, _ = St.solve(src)
    d_obs = ut.reshape(len(c["sources"]), -1)[:, rec.long()].contiguous()
    St.close()
    s0 = torch.from_numpy(c["s_init"]).cuda()

    def step():
        s = s0.clone().requires_grad_(True)
        J = adjoint.misfit(s, omega, grid, src, rec, d_obs, **opts)
        J.backward()
        return J.item(), s.grad

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        J, g = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    line = {
        "metric": "misfit gradients/s (forward + adjoint solves of all shots, gradient)",
        "value": a.steps / el, "unit": "gradients/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"adjoint_{c['nx']}x{c['ny']}_f{c['freq']:g}_shots{len(src)}",
                   "grid": f"{c['nx']}x{c['ny']}", "h_m": c["h"], "freq_hz": c["freq"],
                   "shots": len(src), "receivers": int(rec.numel()), "batched": bool(a.batch),
                   "J": J, "grad_norm": float(g.norm())},
    }
    print(json.dumps(line), flush=True)


def layered_multi_bench(a, torch, H, inputs, prec):
    """Sources x frequencies of the layered model: one step = for every
    frequency, create its handle (the operator depends on the frequency),
    solve all sources in one batched FGMRES, destroy the handle.  Handle set-up
    is inside the timed region (whole-job throughput)."""
    freqs = [float(f) for f in a.freqs.split(",") if f.strip()]
    ws = [inputs.layered(freq=f, nsrc=a.nrhs) for f in freqs]
    kfs = [torch.from_numpy(w.kfield()).cuda() for w in ws]
    bs = [torch.from_numpy(w.sources()).cuda() for w in ws]

    def opts(w):
        return dict(coarse_op=w.coarse_op, coarse_mode=H.CMODE_TOL, coarse_tol=w.coarse_tol,
                    coarse_iters=w.coarse_maxit, coarse_restart=w.coarse_restart,
                    restart=w.restart, tol=w.tol, batch=a.batch, graphs=a.graphs,
                    vc_tail=a.vc_tail)

    def step(precision, keep=False):
        infos, xs = [], []
        for w, kf, b in zip(ws, kfs, bs):
            t = time.perf_counter()
            S = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, k=kf, precision=precision, **opts(w))
            x, info = S.solve(b)
            S.close()
            # progress on stderr (the solve has synchronised already)
            print(f"bench.py: {w.freq:g} Hz, {len(info)} sources, precision {precision}: "
                  f"{time.perf_counter() - t:.2f} s", file=sys.stderr, flush=True)
            infos.append(info)
            if keep:
                xs.append(x)
        return infos, xs

    for _ in range(a.warmup):
        step(prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        infos, _ = step(prec)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if not all(i["converged"] for inf in infos for i in inf):
        print("bench.py: a solve did not converge", file=sys.stderr)
        sys.exit(1)
    nsol = a.nrhs * len(freqs)
    per_f = {f"{f:g}Hz": {"outer_iters": [min(i["outer_iters"] for i in inf),
                                          max(i["outer_iters"] for i in inf)],
                          "inner_iters_sum": sum(i["inner_iters_total"] for i in inf),
                          "relres_max": max(i["relres"] for i in inf)}
             for f, inf in zip(freqs, infos)}
    line = {
        "metric": "Helmholtz solves/s to 1e-6 rel. residual (sources x frequencies, batched)",
        "value": nsol * a.steps / el, "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == H.PREC_FP64 else "f64 (f32 fine-grid V-cycle)",
        "data": "synthetic",
        "config": {"workload": f"layered_{ws[0].nx}x{ws[0].ny}_x{a.nrhs}_f"
                               + "-".join(f"{f:g}" for f in freqs)
                               + ("" if prec == H.PREC_FP64 else "_mixed"),
                   "grid": f"{ws[0].nx}x{ws[0].ny}", "h_m": ws[0].hx, "sources": a.nrhs,
                   "freqs_hz": freqs, "batched": bool(a.batch),
                   "krylov": f"FGMRES({ws[0].restart}) to {ws[0].tol:g}",
                   "coarse_solve": f"GMRES({ws[0].coarse_restart}) to {ws[0].coarse_tol:g}",
                   "per_frequency": per_f},
    }
    if prec != H.PREC_FP64:
        # accuracy against the FP64 solves of the same sources (outside the
        # timed region)
        _, x32 = step(prec, keep=True)
        _, x64 = step(H.PREC_FP64, keep=True)
        d = max(((u - v).reshape(a.nrhs, -1).norm(dim=1) / v.reshape(a.nrhs, -1).norm(dim=1))
                .max().item() for u, v in zip(x32, x64))
        line["config"]["max_rel_diff_to_fp64_solution"] = d
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); "
              "the solve is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2308_06152_amd import helmdefl as H
    from paper_2308_06152_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.workload == "adjoint":
        adjoint_bench(a, torch, H, inputs)
        return
    if a.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.complex128, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "layered" and a.freqs:
        prec = {"fp64": H.PREC_FP64, "mixed": H.PREC_MIXED,
                "mixed_c64basis": H.PREC_MIXED_C64BASIS}[a.precision]
        layered_multi_bench(a, torch, H, inputs, prec)
        return
    if a.workload == "layered":
        w = inputs.layered(freq=a.freq, nsrc=a.nrhs)
    else:
        w = {"large": inputs.large_plain, "small": inputs.small_plain,
             "wedge": inputs.wedge}[a.workload]()
    kf = w.kfield()
    prec = {"fp64": H.PREC_FP64, "mixed": H.PREC_MIXED,
            "mixed_c64basis": H.PREC_MIXED_C64BASIS}[a.precision]
    kt = None if kf is None else torch.from_numpy(kf).cuda()
    nrhs = w.nsrc if w.model == "layered" else 1
    b = torch.from_numpy(w.sources() if nrhs > 1 else w.rhs()).cuda()
    opts = dict(coarse_op=w.coarse_op, coarse_mode=H.CMODE_TOL, coarse_tol=w.coarse_tol,
                coarse_iters=w.coarse_maxit, coarse_restart=w.coarse_restart, restart=w.restart,
                tol=w.tol, precision=prec, batch=a.batch, graphs=a.graphs, vc_tail=a.vc_tail)
    tuned = {}
    if a.autotune != "off":
        from paper_2308_06152_amd import autotune
        grid = (w.nx, w.ny, w.hx, w.hy, w.bc)
        cache = a.tune_cache or autotune.DEFAULT_CACHE
        if a.autotune == "run":
            tuned = autotune.tune(grid, b, opts, k=kt, kconst=w.kconst, cache_path=cache,
                                  retune=True, log=lambda m: print(m, file=sys.stderr))
        else:
            tuned = autotune.lookup(grid, nrhs, opts, kt is not None, cache_path=cache)
        opts.update(tuned)
    S = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, k=kt, kconst=w.kconst, **opts)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        S.solve(b, x)
    # timed region: the solves alone (no kernel timing events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(a.steps):
        _, info = S.solve(b, x)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # second timed region, the same solves with HIP events recorded on the
    # solver's stream around every launch of the roofline kernel
    kclass = H.KERNEL_CLASS_NAMES.index(a.roofline_kernel)
    S.timing_enable(kclass, a.roofline_level)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(a.steps):
        S.solve(b, x)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n_launch, k_ms, k_bytes = S.timing_read()
    S.timing_enable(-1, -1)
    last = infos[-1][0]
    if not all(i["converged"] for step in infos for i in step):
        print("bench.py: a solve did not converge", file=sys.stderr)
        sys.exit(1)
    achieved = (k_bytes / 1e9) / (k_ms / 1e3) if k_ms > 0 else 0.0
    traffic = (measured_traffic(a.roofline_kernel, w.name, opts["coarse_restart"])
               if prec == H.PREC_FP64 and nrhs == 1 else None)
    mixed = prec != H.PREC_FP64
    wname = w.name + {H.PREC_FP64: "", H.PREC_MIXED: "_mixed",
                      H.PREC_MIXED_C64BASIS: "_mixed_c64basis"}[prec]
    line = {
        "metric": METRIC,
        "value": nrhs * a.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if not mixed else "f64 (f32 fine-grid V-cycle"
                  + (", c64 coarse basis)" if prec == H.PREC_MIXED_C64BASIS else ")")),
        "data": "synthetic",
        "config": {
            "workload": wname,
            "grid": f"{w.nx}x{w.ny}",
            "k": w.kconst if kf is None else f"{w.model} model at {w.freq:g} Hz",
            "bc": "sommerfeld" if w.bc == H.BC_SOMMERFELD else "dirichlet",
            "source": "gaussian sigma=2h" if w.source == "gauss" else "point",
            "preconditioner": "APD (Bezier Z, " + ("ReD-Glk2" if w.coarse_op else "Galerkin")
                              + " A_2h) + 1 CSLP V-cycle (1,0.5)"
                              + ({H.PREC_FP64: "", H.PREC_MIXED: ", fine-grid V-cycle in complex64",
                                  H.PREC_MIXED_C64BASIS: ", fine-grid V-cycle in complex64, "
                                                         "complex64 coarse basis"}[prec]),
            "krylov": f"FGMRES({w.restart}) to {w.tol:g}",
            "coarse_solve": f"GMRES({opts['coarse_restart']}) to {w.coarse_tol:g}",
            "outer_iters": last["outer_iters"], "inner_iters_total": last["inner_iters_total"],
            "relres": last["relres"], "graphs": bool(opts["graphs"]), "vc_tail": opts["vc_tail"],
            "autotuned": tuned or None,
            **({"nrhs": nrhs, "batched": bool(a.batch),
                "outer_iters_max": max(i["outer_iters"] for i in infos[-1]),
                "inner_iters_sum": sum(i["inner_iters_total"] for i in infos[-1]),
                "relres_max": max(i["relres"] for i in infos[-1])} if nrhs > 1 else {}),
        },
        "roofline": {
            "kernel": a.roofline_kernel, "level": a.roofline_level, "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "launches": n_launch, "avg_launch_us": 1e3 * k_ms / max(n_launch, 1),
            "alg_bytes_per_launch": k_bytes / max(n_launch, 1),
            "ms_per_step_with_events": 1e3 * (t3 - t2) / a.steps,
        },
    }
    if mixed:
        # accuracy of the mixed-precision solution: against the FP64 solve of
        # the same workload (the FP64 path matches the oracle per solve)
        S64 = H.Solver(w.nx, w.ny, w.hx, w.hy, w.bc, k=kt, kconst=w.kconst,
                       **dict(opts, precision=H.PREC_FP64))
        x64, info64 = S64.solve(b)
        S64.close()
        xs, xr = x.reshape(nrhs, -1), x64.reshape(nrhs, -1)
        diff = ((xs - xr).norm(dim=1) / xr.norm(dim=1)).max().item()
        line["config"]["fp64_reference"] = {
            "outer_iters": info64[0]["outer_iters"],
            "inner_iters_total": info64[0]["inner_iters_total"],
            "relres": info64[0]["relres"],
            "max_rel_diff_to_fp64_solution": diff,
        }
    if not a.no_cpu_baseline:
        if w.nx * w.ny <= 300 * 300:
            line["cpu_baseline"] = cpu_baseline_full(w, S.opts.coarsest_nodes,
                                                     opts["coarse_restart"])
        else:
            line["cpu_baseline"] = cpu_baseline(w, last, S.opts.coarsest_nodes,
                                                opts["coarse_restart"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
