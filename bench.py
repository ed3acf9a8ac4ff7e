"""Benchmark: ADR amplitude solves on one MI355X.

Metric: Mpoints/s of a whole solve (FGMRES(5) + V-cycle from a zero guess to true
relative residual <= 1e-6, then the wavefield u = a exp(-i w tau)), mixed precision
(complex-FP32 V-cycle, FP64 outer) vs FP64, on the 3D 129^3 linear-gradient workload
(v = 1.5 + 0.8 z km/s on a 1 km cube, analytic travel time, source at (0.5, 0.5, 0.1) km,
10 points per wavelength).  Setup (coefficients, Galerkin hierarchy, coarsest inverse)
is timed separately.  Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line.  --gpus N with N > 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TOL = 1e-6
TIMER_LAUNCHES = 65536   # launches one adr_timer_start can time


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="3d_129",
                    choices=["3d_129", "2d_129", "3d_65", "3d_257", "batch_2d", "adjoint_3d_193", "compare_3d_129"])
    ap.add_argument("--adjoint-n", type=int, default=193, help="grid size of the adjoint workload")
    ap.add_argument("--fm-workers", type=int, default=8, help="CPU processes for fast marching")
    ap.add_argument("--streams", type=int, default=4, help="streams of the batched-shot solve")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="GPU_MAX_HW_QUEUES for this process (set before the GPU is initialized; <= 32)")
    ap.add_argument("--cycle", default="v", choices=["v", "k"], help="V-cycle or Krylov cycle preconditioner")
    ap.add_argument("--kcycle-levels", type=int, default=0,
                    help="Krylov cycle: flexible-GMRES coarse solves on coarse levels 1..K only (0 = all)")
    ap.add_argument("--shift", type=float, default=0.2,
                    help="compare_3d_129: shifted-Laplacian alpha of the preconditioner")
    ap.add_argument("--batch-maxit", type=int, default=3000, help="FGMRES iteration cap per shot (batch)")
    ap.add_argument("--no-looped", action="store_true", help="batch: skip the one-shot-at-a-time comparison")
    ap.add_argument("--no-batch", action="store_true", help="default line: skip the batched-shot leg")
    ap.add_argument("--batch-merge", type=int, default=2, choices=[0, 1, 2],
                    help="batch: 0 = one group per grid shape, 1 = one merged group, 2 = both")
    ap.add_argument("--mixed-only", action="store_true", help="with --profile-only: skip the FP64 solves")
    ap.add_argument("--no-graph", action="store_true", help="launch the cycles eagerly (no hipGraph)")
    ap.add_argument("--pipeline-max-nodes", type=int, default=None,
                    help="coarse levels up to this many nodes use the pipelined relaxation "
                         "(0 = off; default: the library's, every coarse level)")
    ap.add_argument("--coarse-split", type=int, default=0, choices=[0, 1, 4],
                    help="Galerkin-apply variant on every coarse level (0 = timed at setup)")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning-table", default=None, metavar="PATH",
                    help="read the Galerkin-apply autotuner's table from PATH before any setup (fixes the "
                         "variant choices, e.g. for counter runs of the same configuration)")
    ap.add_argument("--tuning-table-out", default=None, metavar="PATH",
                    help="write the autotuner's table to PATH at the end")
    ap.add_argument("--no-257", action="store_true",
                    help="default workload: skip the 3D 257^3 leg that carries the HBM roofline")
    ap.add_argument("--cpu-sample-iters", type=int, default=60,
                    help="iteration cap of the CPU oracle solve (default: enough for the 129^3 workload)")
    ap.add_argument("--cpu-sample-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--profile-only", action="store_true",
                    help="setup + warmup + timed steps only (for rocprofv3 runs)")
    return ap.parse_args()


KERNEL_SOURCES = [os.path.join(ROOT, "paper_1712_06091_amd", "csrc", f)
                  for f in ("adr_kernels.hip", "adr_kernels.hpp", "adr_common.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pipe_opt(args):
    """Option overrides for --pipeline-max-nodes (none: the library default) and
    --kcycle-levels."""
    o = {"kcycle_levels": args.kcycle_levels}
    if args.pipeline_max_nodes is not None:
        o["pipeline_max_nodes"] = args.pipeline_max_nodes
    return o


def measured_traffic(workload):
    """HBM bytes from the committed counter summary of this workload (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy): {"level1": per level-1 Galerkin apply, "vcycle":
    per V-cycle}, or None when there is no summary or the kernel sources changed since
    it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.strip().startswith("- `"):
                k, v = line.strip()[3:].split("`", 1)
                vals[k] = v.split(":", 1)[1].strip().strip("`")
    if vals.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    return {"level1": float(vals["level1_traffic_bytes_per_launch"]), "vcycle": float(vals["vcycle_traffic_bytes"])}


def make_workload(name):
    from paper_1712_06091_amd import workloads as W
    if name == "3d_129":
        return W.config_3d_129()
    if name == "2d_129":
        return W.config_2d_129()
    if name == "3d_257":
        return W.config_3d_257()
    return W.linear_gradient(65, ndim=3, name="3d_65_linear_gradient")


# --------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle (NumPy/SciPy, one thread) on a bounded sample
# --------------------------------------------------------------------------------------
def cpu_sample_child(args):
    """Runs in a child process with every BLAS/OpenMP pool limited to one thread: the FP64
    oracle's own FGMRES(5) + V-cycle on the full workload, from zero until the true relative
    residual reaches the benchmark tolerance (or --cpu-sample-iters iterations)."""
    from oracle import krylov
    from oracle import solve as osolve
    wl = make_workload(args.workload)
    t0 = time.perf_counter()
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy()
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega).ravel()
    t1 = time.perf_counter()
    _, info = krylov.fgmres(lambda v: p.H2up @ v, qh, precond=hier.vcycle, restart=5, tol=TOL,
                            maxit=args.cpu_sample_iters)
    t2 = time.perf_counter()
    print(json.dumps({"setup_s": t1 - t0, "iters": info["iters"], "solve_s": t2 - t1,
                      "relres": info["relres"]}))


def cpu_baseline(args, nodes, iters_needed):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample-child", "--workload", args.workload,
           "--cpu-sample-iters", str(args.cpu_sample_iters)]
    out = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, check=True, cwd=ROOT)
    r = json.loads(out.stdout.decode().strip().splitlines()[-1])
    done = r["relres"] <= TOL
    per_iter = r["solve_s"] / max(r["iters"], 1)
    t = r["solve_s"] if done else per_iter * iters_needed
    if done:
        sample = (f"FP64 oracle FGMRES(5) + V-cycle (NumPy/SciPy, one thread) on the full workload: a whole solve "
                  f"from zero to true relative residual {r['relres']:.2e} <= {TOL:g} in {r['iters']} iterations, "
                  f"{r['solve_s']:.1f} s (setup {r['setup_s']:.1f} s not counted)")
    else:
        sample = (f"FP64 oracle FGMRES(5) + V-cycle (NumPy/SciPy, one thread) on the full workload: {r['iters']} "
                  f"iterations in {r['solve_s']:.1f} s ({per_iter:.2f} s/iteration, setup {r['setup_s']:.1f} s not "
                  f"counted), scaled to the {iters_needed} iterations the FP64 GPU solve needs to reach {TOL:g}")
    return {"value": nodes / t / 1e6, "unit": "Mpoints/s", "cores": 1, "kind": "oracle", "sample": sample,
            "whole_solve": done, **host_cpu()}


# --------------------------------------------------------------------------------------
# GPU
# --------------------------------------------------------------------------------------
def copy_probe(args):
    """A plain device-to-device copy of a known size (reads and writes args.copy_probe MiB
    once each): the reference dispatch for scaling the HBM byte counters."""
    import torch
    n = int(args.copy_probe * 2 ** 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 8 * n}))


def run_adjoint(args):
    """Misfit gradient: 16 sources on an n^3 smooth random medium, a 64 x 64 receiver plane
    on the top face, data from a seeded 5% kappa^2 perturbation; one step = J and
    dJ/dkappa^2 through the autograd Function (16 forward + 16 adjoint solves to 1e-6,
    context setup included, since tau differs per source)."""
    import numpy as np

    from paper_1712_06091_amd import workloads as W
    t0 = time.perf_counter()
    wl = W.adjoint_3d(args.adjoint_n, workers=args.fm_workers)   # CPU only, before the GPU is touched
    log(f"adjoint workload {wl.name}: {len(wl.sources)} sources, {wl.receivers.size} receivers, "
        f"inputs in {time.perf_counter() - t0:.1f} s")
    import torch

    from paper_1712_06091_amd import adr, misfit
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(a, dtype=dt, device=dev)
    k2, k2t, gam = t(wl.kappa2, torch.float64), t(wl.kappa2_true, torch.float64), t(wl.gamma, torch.float64)
    taus = [t(x, torch.float64) for x in wl.taus]
    rec = t(wl.receivers, torch.int32)
    opts = adr.default_options(prec="mixed", cycle=args.cycle)
    N = int(np.prod(wl.shape))
    d_obs = []
    for tau, src in zip(taus, wl.sources):
        c = adr.Context(k2t, tau, gam, wl.h, wl.omega, src, options=opts)
        a, st = c.solve(misfit.point_source(wl.shape, src, wl.h, dev), tol=1e-8, maxit=1000)
        if st["status"] != adr.ADR_OK:
            raise RuntimeError(f"data solve did not converge: {st}")
        d_obs.append(c.wavefield(a).reshape(-1)[rec.long()].clone())
        c.close()
    log("observed data done")

    def step(stats=None):
        kp = k2.clone().requires_grad_(True)
        J = misfit.receiver_misfit(kp, gam, taus, wl.sources, wl.h, wl.omega, rec, d_obs, options=opts, tol=TOL,
                                   stats=stats)
        J.backward()
        return float(J.detach()), kp.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times, stats = [], []
    for _ in range(args.steps):
        stats = []
        t1 = time.perf_counter()
        J, g = step(stats)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        log(f"gradient step {times[-1]:.1f} s, J = {J:.4e}")
    ms = 1e3 * sum(times) / len(times)
    fw = [s["outer_iters"] for k, s in stats if k == "forward"]
    ad = [s["outer_iters"] for k, s in stats if k == "adjoint"]
    solve_ms = sum(s["solve_ms"] for _, s in stats)
    setup_ms = sum(s["setup_ms"] for k, s in stats if k == "forward")
    nsolve = len(stats)
    out = {
        "metric": "ADR amplitude solves: Mpoints/s to 1e-6 residual (misfit gradient, forward + adjoint)",
        "value": nsolve * N / (ms * 1e-3) / 1e6, "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 V-cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.shape), "sources": len(wl.sources),
                   "receivers": int(wl.receivers.size), "tol": TOL, "cycle": args.cycle, "omega": wl.omega},
        "J": J, "grad_norm": float(g.norm()),
        "forward_iters": {"min": min(fw), "max": max(fw), "total": sum(fw)},
        "adjoint_iters": {"min": min(ad), "max": max(ad), "total": sum(ad)},
        "solve_ms_total": solve_ms, "setup_ms_total": setup_ms,
        "solve_only_value": nsolve * N / (solve_ms * 1e-3) / 1e6,
    }
    print(json.dumps(out))


def looped_batch(shots, qs, outs, opts, maxit):
    """The same shots one after another through adr_solve on the default stream; returns
    (ms, total iterations, largest final true relative residual)."""
    import torch

    from paper_1712_06091_amd import adr
    ctxs = [adr.Context(s["kappa2"], s["tau"], s["gamma"], s["h"], s["omega"], s["src"], options=opts)
            for s in shots]
    for c, q, a in zip(ctxs, qs, outs):
        c.solve(q, tol=TOL, maxit=maxit, out=a)
    torch.cuda.synchronize()
    log("looped warm-up done")
    t0 = time.perf_counter()
    iters, worst = 0, 0.0
    for c, q, a in zip(ctxs, qs, outs):
        _, s1 = c.solve(q, tol=TOL, maxit=maxit, out=a)
        iters += s1["outer_iters"]
        worst = max(worst, s1["relres"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    for c in ctxs:
        c.close()
    return ms, iters, worst


def batched(shots, qs, outs, opts, args, maxit):
    """One lockstep batched solve of every shot; returns (ms per batch, stats, setup s)."""
    import torch

    from paper_1712_06091_amd import adr
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    b = adr.Batch(shots, options=opts, nstreams=args.streams)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - s0
    for _ in range(args.warmup):
        b.solve(qs, outs, tol=TOL, maxit=maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, stats = b.solve(qs, outs, tol=TOL, maxit=maxit)
        if st != adr.ADR_OK:
            bad = [(i, s["outer_iters"], s["relres"]) for i, s in enumerate(stats) if not s["relres"] <= TOL]
            raise RuntimeError(f"batched solve did not converge within {maxit} iterations: {bad[:8]}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    b.close()
    return ms, stats, setup_s


def batch_figures(wls, args, merges, steps, warmup, looped=True):
    """Batched solves of the shots ``wls`` to 1e-6 (mixed and FP64; one group per grid
    shape and/or one merged group, per ``merges``) and, with ``looped``, the same shots
    solved one after another in FP64 (adr_solve).  Returns the legs' figures."""
    import numpy as np
    import torch

    from paper_1712_06091_amd import adr

    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    shots = [{"kappa2": t(w.kappa2, torch.float64), "tau": t(w.tau, torch.float64),
              "gamma": t(w.gamma, torch.float64), "h": w.h, "omega": w.omega, "src": w.src} for w in wls]
    qs = [t(w.rhs(), torch.complex128) for w in wls]
    outs = [torch.empty(w.shape, dtype=torch.complex128, device=dev) for w in wls]
    nodes = sum(w.nodes for w in wls)
    maxit = args.batch_maxit
    bargs = argparse.Namespace(**vars(args))
    bargs.steps, bargs.warmup = steps, warmup
    legs = {}
    for merge in merges:
        for prec in ("mixed", "fp64"):
            opts = adr.default_options(prec=prec, cycle=args.cycle, batch_merge=merge, **pipe_opt(args))
            ms, stats, setup_s = batched(shots, qs, outs, opts, bargs, maxit)
            its = sorted(s["outer_iters"] for s in stats)
            by_size = {}
            for w, st_ in zip(wls, stats):
                by_size[w.shape[0]] = max(by_size.get(w.shape[0], 0), st_["outer_iters"])
            key = prec + ("_merged" if merge else "")
            legs[key] = {"value": nodes / (ms * 1e-3) / 1e6, "ms_per_step": ms, "setup_s": setup_s,
                         "outer_iters": sum(its),
                         "outer_iters_per_shot": {"min": its[0], "median": its[len(its) // 2], "max": its[-1]},
                         "outer_iters_max_by_size": {str(k): v for k, v in sorted(by_size.items())},
                         "final_relres_max": max(s["relres"] for s in stats)}
            log(f"batched {key}: {ms:.1f} ms per batch; iterations min {its[0]} median {its[len(its) // 2]} "
                f"max {its[-1]}")
    lp = None
    if looped:
        opts = adr.default_options(prec="fp64", cycle=args.cycle, **pipe_opt(args))
        ms_loop, iters_loop, worst = looped_batch(shots, qs, outs, opts, maxit)
        lp = {"precision": "fp64", "value": nodes / (ms_loop * 1e-3) / 1e6, "ms": ms_loop,
              "outer_iters": iters_loop, "final_relres_max": worst}
        log(f"looped fp64: {ms_loop:.1f} ms")
    m = legs["mixed"] if "mixed" in legs else legs["mixed_merged"]
    return {
        "shots": len(wls), "nodes": nodes, "sizes": sorted({w.shape[0] for w in wls}), "tol": TOL,
        "steps": steps, "warmup": warmup,
        "batched_mixed": legs.get("mixed"), "batched_fp64": legs.get("fp64"),
        "batched_mixed_merged": legs.get("mixed_merged"), "batched_fp64_merged": legs.get("fp64_merged"),
        "looped_fp64": lp,
        "batched_mixed_over_looped_fp64": None if lp is None else lp["ms"] / m["ms_per_step"],
        "batched_fp64_over_looped_fp64": (None if lp is None or "fp64" not in legs
                                          else lp["ms"] / legs["fp64"]["ms_per_step"]),
    }


def run_batch(args):
    """64 2D shots (sizes from {257^2, 513^2, 1025^2}, random media, fast-marching tau):
    lockstep batched solves over several streams in mixed precision (the value) and in
    FP64, against the same shots solved one after another in FP64 (adr_solve), all to the
    same true relative residual 1e-6."""
    from paper_1712_06091_amd import workloads as W

    wls = W.batch_2d(workers=8)
    log(f"batch: {len(wls)} shots, {sum(w.nodes for w in wls) / 1e6:.1f} M nodes")
    merges = {0: (0,), 1: (1,), 2: (0, 1)}[args.batch_merge]
    fig = batch_figures(wls, args, merges, args.steps, args.warmup, looped=not args.no_looped)
    m = fig["batched_mixed"] or fig["batched_mixed_merged"]
    out = {
        "metric": "ADR amplitude solves: Mpoints/s to 1e-6 residual (batched shots)",
        "value": m["value"], "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 V-cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": "batch_2d_64_shots", "shots": fig["shots"], "nodes": fig["nodes"],
                   "sizes": fig["sizes"], "streams": args.streams, "tol": TOL,
                   "cycle": args.cycle, "maxit": args.batch_maxit,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "0")) or None},
        "outer_iters": m["outer_iters"],
    }
    out.update({k: v for k, v in fig.items() if k.startswith(("batched", "looped"))})
    print(json.dumps(out))


def run_compare(args):
    """The three discretizations of the paper's performance tables (Sec. 4.2) on the 3D
    129^3 linear-gradient medium and source: standard Helmholtz with the shifted-Laplacian
    preconditioner (alpha = --shift), the ADR-central system by the two-stage solve, and
    the ADR-upwind system; FGMRES(5), the --cycle preconditioner, to 1e-6."""
    import numpy as np
    import torch

    from paper_1712_06091_amd import adr, workloads as W

    dev = torch.device("cuda:0")
    wl = W.config_3d_129()
    N = wl.nodes
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    k2, tau, gam = t(wl.kappa2, torch.float64), t(wl.tau, torch.float64), t(wl.gamma, torch.float64)
    q = t(wl.rhs(), torch.complex128)
    out = torch.empty(wl.shape, dtype=torch.complex128, device=dev)
    maxit = 2000

    def timed(solve_once):
        for _ in range(args.warmup):
            solve_once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            its, st = solve_once()
            if st["status"] != adr.ADR_OK or not st["relres"] <= TOL:
                raise RuntimeError(f"solve did not converge: {st}")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        return {"value": N / (ms * 1e-3) / 1e6, "ms_per_step": ms, "outer_iters": its}

    res = {}
    for name, tau_arg, alpha in (("standard", None, args.shift), ("adr_upwind", tau, 0.0)):
        ctx = adr.Context(k2, tau_arg, gam, wl.h, wl.omega, wl.src,
                          options=adr.default_options(prec="mixed", cycle=args.cycle, shift_alpha=alpha))

        def once(ctx=ctx):
            _, st = ctx.solve(q, tol=TOL, maxit=maxit, out=out)
            return st["outer_iters"], st
        res[name] = timed(once)
        log(f"{name}: {res[name]['ms_per_step']:.1f} ms/solve, {res[name]['outer_iters']} iterations")
        ctx.close()
    o1, o2 = adr.two_stage_options("mixed")
    o1.cycle = o2.cycle = adr.ADR_CYCLE_K if args.cycle == "k" else adr.ADR_CYCLE_V
    o2.shift_alpha = args.shift
    c1 = adr.Context(k2, tau, gam, wl.h, wl.omega, wl.src, options=o1)
    c2 = adr.Context(k2, tau, gam, wl.h, wl.omega, wl.src, options=o2)

    def once2():
        _, s1, s2 = adr.solve_two_stage(c1, c2, q, tol=TOL, maxit=maxit, out=out)
        return [s1["outer_iters"], s2["outer_iters"]], s2
    res["adr_central_two_stage"] = timed(once2)
    log(f"adr_central_two_stage: {res['adr_central_two_stage']['ms_per_step']:.1f} ms/solve, "
        f"{res['adr_central_two_stage']['outer_iters']} iterations (stage 1, stage 2)")
    c1.close()
    c2.close()
    up = res["adr_upwind"]
    print(json.dumps({
        "metric": "Discretization comparison, Mpoints/s to 1e-6 residual (value: ADR upwind)",
        "value": up["value"], "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": up["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": "compare_3d_129_linear_gradient", "grid": list(wl.shape), "nodes": N,
                   "omega": wl.omega, "tol": TOL, "restart": 5, "shift_alpha": args.shift, "cycle": args.cycle},
        "outer_iters": up["outer_iters"],
        "standard_shifted_laplacian": res["standard"],
        "adr_central_two_stage": res["adr_central_two_stage"],
        "adr_upwind": up,
    }))


def host_cpu():
    """Host cores and model (the GPU machine's host, read at run time)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cores": os.cpu_count(), "host_cpu": model}


def gpu_tensors(wl):
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    return (t(wl.kappa2, torch.float64), t(wl.tau, torch.float64), t(wl.gamma, torch.float64),
            t(wl.rhs(), torch.complex128))


def make_ctx(wl, tensors, prec, args):
    from paper_1712_06091_amd import adr
    k2, tau, gam, _ = tensors
    return adr.Context(k2, tau, gam, wl.h, wl.omega, wl.src,
                       options=adr.default_options(prec=prec, cycle=args.cycle, use_graph=0 if args.no_graph else 1,
                                                   coarse_split=args.coarse_split, **pipe_opt(args)))


def solve_step(ctx, q, a, u, tol=TOL, maxit=3000):
    """One benchmark step: a whole solve from zero to tol, then the wavefield."""
    from paper_1712_06091_amd import adr
    _, st = ctx.solve(q, tol=tol, maxit=maxit, out=a)
    ctx.wavefield(a, out=u)
    if st["status"] != adr.ADR_OK or not st["relres"] <= tol:
        raise RuntimeError(f"solve did not converge: {st}")
    return st


def timed_solves(ctx, q, a, u, steps, warmup):
    import torch
    for _ in range(warmup):
        solve_step(ctx, q, a, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = [solve_step(ctx, q, a, u) for _ in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, sts


def level1_roofline(ctx, q, a, u, workload, cache_note=None):
    """The dominant kernel, the 81/21-point Galerkin apply on level 1 (plain launches and
    the pipelined relaxation steps that carry it), timed by the library's HIP events on the
    context stream over one whole mixed solve."""
    ctx.timer_start("coarse_apply", 1)
    solve_step(ctx, q, a, u)
    ms, n, by = ctx.timer_stop()
    avg_ms = ms / max(n, 1)
    avg_bytes = by / max(n, 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    shape, S = ctx.level_info(1)
    traffic = measured_traffic(workload)
    out = {"bound": "hbm", "workload": workload,
           "kernel": (f"k_coarse_apply + k_pipe_step (level 1, {'x'.join(map(str, shape))}, {S}-point Galerkin "
                      "stencil, c64)"),
           "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
           "traffic": traffic["level1"] if traffic else None, "avg_launch_ms": avg_ms, "launches": n,
           "algorithmic_bytes_per_launch": avg_bytes}
    if cache_note:
        out["note"] = cache_note
    return out


def vcycle_figures(ctx, shape, workload, reps=20):
    """One V-cycle: algorithmic bytes summed over its kernel classes (library HIP events),
    time by torch events around `reps` cycles on the current stream (the context's)."""
    import torch
    from paper_1712_06091_amd import adr
    classes = list(adr.TIMER_KINDS)
    r = torch.randn(shape, dtype=torch.complex128, device="cuda:0")
    z = torch.empty_like(r)
    vc_bytes = 0.0
    for cls in classes[:5]:
        ctx.timer_start(cls)
        ctx.vcycle(r, out=z)
        _, _, by = ctx.timer_stop()
        vc_bytes += by
    for _ in range(3):
        ctx.vcycle(r, out=z)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.vcycle(r, out=z)
    e1.record()
    torch.cuda.synchronize()
    vc_ms = e0.elapsed_time(e1) / reps
    traffic = measured_traffic(workload)
    gbps = vc_bytes / (vc_ms * 1e-3) / 1e9
    return {"ms": vc_ms, "algorithmic_bytes": vc_bytes, "GBps": gbps, "frac": gbps / HBM_PEAK_GBPS,
            "traffic": traffic["vcycle"] if traffic else None}


def accuracy(ctx64, q, a_mixed, a_fp64):
    """Errors of the benchmark results against an FP64 solve to 1e-10 (whose true residual
    the GPU tests check with the oracle's matrix)."""
    import torch
    ref, st = ctx64.solve(q, tol=1e-10, maxit=5000)
    nr = torch.linalg.vector_norm(ref).item()
    return {"reference": "FP64 GPU solve to true relative residual 1e-10", "reference_relres": st["relres"],
            "mixed_rel_l2": torch.linalg.vector_norm(a_mixed - ref).item() / nr,
            "fp64_rel_l2": torch.linalg.vector_norm(a_fp64 - ref).item() / nr}


def tuning_table():
    """The autotuner's choices so far (written by the library, read back)."""
    import tempfile

    from paper_1712_06091_amd import adr
    with tempfile.NamedTemporaryFile("r", suffix=".txt") as fh:
        adr.tuning_table_write(fh.name)
        rows = [l.split() for l in fh.read().splitlines() if l and not l.startswith("#")]
    return [{"ndim": int(r[0]), "shape": [int(r[1]), int(r[2]), int(r[3])], "real_bytes": int(r[4]),
             "variant": int(r[5]), "slabs": int(r[6]), "ms_per_8": float(r[7])} for r in rows]


def hbm_leg(args):
    """3D 257^3 random medium (fast-marching tau): where the working set exceeds the
    256 MB Infinity Cache, so the level-1 apply and the V-cycle are HBM-bound.  A few whole
    solves in each precision, the level-1 roofline, the V-cycle fraction."""
    import torch
    wl = make_workload("3d_257")
    tens = gpu_tensors(wl)
    q = tens[3]
    a = torch.empty(wl.shape, dtype=torch.complex128, device="cuda:0")
    u = torch.empty_like(a)
    a64 = torch.empty_like(a)
    s0 = time.perf_counter()
    ctx = make_ctx(wl, tens, "mixed", args)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - s0) * 1e3
    ms_m, st_m = timed_solves(ctx, q, a, u, 2, 1)
    log(f"3d_257 mixed: {ms_m:.1f} ms/solve, {st_m[-1]['outer_iters']} iterations")
    levels = ctx.num_levels
    splits = [ctx.level_split(l) for l in range(1, levels - 1)]
    roof = level1_roofline(ctx, q, a, u, "3d_257")
    vc = vcycle_figures(ctx, wl.shape, "3d_257")
    log(f"3d_257 level-1 apply {roof['avg_launch_ms'] * 1e3:.1f} us/launch ({roof['frac']:.3f}); "
        f"V-cycle {vc['ms']:.3f} ms ({vc['frac']:.3f})")
    ctx.close()
    kc = None
    if args.cycle == "v":
        # The Krylov cycle on the same problem, its flexible-GMRES coarse solves on coarse
        # levels 1-2 (the fastest variant measured at this size).
        ka = argparse.Namespace(**{**vars(args), "cycle": "k", "kcycle_levels": 2})
        ck = make_ctx(wl, tens, "mixed", ka)
        ms_k, st_k = timed_solves(ck, q, a, u, 1, 1)
        ck.close()
        kc = {"value": wl.nodes / (ms_k * 1e-3) / 1e6, "ms_per_step": ms_k, "outer_iters": st_k[-1]["outer_iters"],
              "final_relres": st_k[-1]["relres"], "kcycle_levels": 2}
        log(f"3d_257 mixed Krylov cycle: {ms_k:.1f} ms/solve, {st_k[-1]['outer_iters']} iterations")
    # The travel time itself on the GPU (factored-eikonal sweeps) against the CPU fast
    # marching that produced the workload's tau.
    from paper_1712_06091_amd import adr
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    tau_gpu, sweeps = adr.eikonal(tens[0], wl.h, wl.src)
    torch.cuda.synchronize()
    eik = {"gpu_ms": (time.perf_counter() - e0) * 1e3, "sweeps": sweeps, "cpu_fast_marching_s": wl.extra.get("fm_s"),
           "max_abs_diff_vs_fast_marching": torch.max(torch.abs(tau_gpu - tens[1])).item(),
           "median_abs_diff_vs_fast_marching": torch.median(torch.abs(tau_gpu - tens[1])).item(),
           "max_tau": torch.max(tens[1]).item()}
    del tau_gpu
    log(f"3d_257 GPU eikonal: {eik['gpu_ms']:.1f} ms, {sweeps} sweeps (CPU fast marching {eik['cpu_fast_marching_s']} s)")
    c64 = make_ctx(wl, tens, "fp64", args)
    ms_d, st_d = timed_solves(c64, q, a64, u, 1, 0)
    log(f"3d_257 fp64: {ms_d:.1f} ms/solve, {st_d[-1]['outer_iters']} iterations")
    acc = accuracy(c64, q, a, a64)
    c64.close()
    N = wl.nodes
    return {"workload": wl.name, "grid": list(wl.shape), "nodes": N, "omega": wl.omega, "levels": levels,
            "coarse_splits": splits,
            "value": N / (ms_m * 1e-3) / 1e6, "ms_per_step": ms_m, "outer_iters": st_m[-1]["outer_iters"],
            "final_relres": st_m[-1]["relres"],
            "fp64": {"value": N / (ms_d * 1e-3) / 1e6, "ms_per_step": ms_d, "outer_iters": st_d[-1]["outer_iters"]},
            "mixed_over_fp64": ms_d / ms_m, "accuracy": acc, "setup_ms": setup_ms, "vcycle": vc,
            "roofline": roof, "kcycle_mixed": kc, "eikonal": eik}


def main():
    args = parse()
    if args.hw_queues:
        if not 1 <= args.hw_queues <= 32:
            print("--hw-queues must be in [1, 32]", file=sys.stderr)
            sys.exit(2)
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.cpu_sample_child:
        cpu_sample_child(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU shot sharding is not implemented).", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args)
        return
    if args.workload == "batch_2d":
        run_batch(args)
        return
    if args.workload == "adjoint_3d_193":
        run_adjoint(args)
        return
    if args.workload == "compare_3d_129":
        run_compare(args)
        return

    batch_wls = None
    if args.workload == "3d_129" and not args.no_batch and not args.profile_only:
        # The batched-shot leg's inputs, with the fast marching in forked processes before
        # anything initializes the GPU.
        from paper_1712_06091_amd import workloads as W
        batch_wls = W.batch_2d(workers=8)
        log(f"batch leg inputs: {len(batch_wls)} shots")

    import torch

    from paper_1712_06091_amd import adr

    if args.tuning_table:
        log(f"tuning table: {adr.tuning_table_read(args.tuning_table)} entries from {args.tuning_table}")
    wl = make_workload(args.workload)
    N = wl.nodes
    tens = gpu_tensors(wl)
    q = tens[3]
    a = torch.empty(wl.shape, dtype=torch.complex128, device="cuda:0")
    a64 = torch.empty_like(a)
    u = torch.empty_like(a)
    torch.cuda.synchronize()

    ctxs, setup_ms = {}, {}
    for prec in (("mixed",) if args.mixed_only else ("mixed", "fp64")):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        ctxs[prec] = make_ctx(wl, tens, prec, args)
        torch.cuda.synchronize()
        setup_ms[prec] = (time.perf_counter() - s0) * 1e3
        log(f"setup {prec}: {setup_ms[prec]:.0f} ms, {ctxs[prec].num_levels} levels")

    ms_mixed, st_mixed = timed_solves(ctxs["mixed"], q, a, u, args.steps, args.warmup)
    log(f"mixed: {ms_mixed:.2f} ms/solve, {st_mixed[-1]['outer_iters']} iterations")
    if args.profile_only and args.mixed_only:
        print(json.dumps({"ms_mixed": ms_mixed, "outer_iters": st_mixed[-1]["outer_iters"],
                          "levels": ctxs["mixed"].num_levels}))
        return
    ms_fp64, st_fp64 = timed_solves(ctxs["fp64"], q, a64, u, max(1, min(args.steps, 3)), 1)
    log(f"fp64: {ms_fp64:.2f} ms/solve, {st_fp64[-1]['outer_iters']} iterations")
    if args.profile_only:
        print(json.dumps({"ms_mixed": ms_mixed, "ms_fp64": ms_fp64}))
        return

    # Kernel-class breakdown of one mixed solve (HIP events around each launch of a class,
    # on the context stream).
    ctx = ctxs["mixed"]
    breakdown = {}
    for cls in adr.TIMER_KINDS:
        ctx.timer_start(cls)
        solve_step(ctx, q, a, u)
        ms, n, by = ctx.timer_stop()
        breakdown[cls] = {"ms": ms, "launches": n, "bytes": by}
    workload_key = args.workload
    cache_note = None
    if args.workload == "3d_129":
        cache_note = ("cache-resident: the level-1 planes (178 MB) fit in the 256 MB Infinity Cache, so this is "
                      "not an HBM figure; the HBM roofline is the 3D 257^3 one")
    roof = level1_roofline(ctx, q, a, u, workload_key, cache_note)
    vc = vcycle_figures(ctx, wl.shape, workload_key)
    log(f"breakdown done; level-1 apply {roof['avg_launch_ms'] * 1e3:.1f} us/launch; V-cycle {vc['ms']:.3f} ms")
    acc = accuracy(ctxs["fp64"], q, a, a64)
    log(f"accuracy vs FP64 1e-10: mixed {acc['mixed_rel_l2']:.2e}, fp64 {acc['fp64_rel_l2']:.2e}")

    iters_m = st_mixed[-1]["outer_iters"]
    iters_d = st_fp64[-1]["outer_iters"]
    value = N / (ms_mixed * 1e-3) / 1e6
    fp64_value = N / (ms_fp64 * 1e-3) / 1e6
    out = {
        "metric": "ADR amplitude solves: Mpoints/s to 1e-6 residual, mixed vs FP64; V-cycle HBM GB/s",
        "value": value,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 V-cycle / c128 FGMRES",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.shape), "nodes": N, "omega": wl.omega,
                   "tol": TOL, "restart": 5, "levels": ctx.num_levels, "precision": "mixed", "cycle": args.cycle,
                   "coarse_splits": [ctx.level_split(l) for l in range(1, ctx.num_levels - 1)]},
        "fp64": {"value": fp64_value, "ms_per_step": ms_fp64, "outer_iters": iters_d},
        "mixed_over_fp64": value / fp64_value,
        "outer_iters": iters_m,
        "final_relres": st_mixed[-1]["relres"],
        "accuracy": acc,
        "setup_ms": setup_ms,
        "vcycle": vc,
        "roofline": roof,
        "breakdown_ms": {c: round(v["ms"], 4) for c, v in breakdown.items()},
        "breakdown_launches": {c: v["launches"] for c, v in breakdown.items()},
        "breakdown_truncated": [c for c, v in breakdown.items() if v["launches"] >= TIMER_LAUNCHES],
    }
    for c in ctxs.values():
        c.close()
    if args.workload == "3d_129" and not args.no_257:
        # The HBM roofline claim: the same kernels where the working set exceeds the cache.
        leg = hbm_leg(args)
        out["roofline_3d_129"] = out["roofline"]
        out["vcycle_3d_129"] = out["vcycle"]
        out["roofline"] = leg.pop("roofline")
        out["vcycle"] = leg.pop("vcycle")
        out["hbm_3d_257"] = leg
    if batch_wls is not None:
        # Config 4: 64 2D shots, batched (one group per grid shape) in mixed precision and
        # FP64 against the same shots solved one after another in FP64; one timed batch each.
        out["batch_2d_64"] = batch_figures(batch_wls, args, (0,), 1, 0, looped=True)
    out["tuning_table"] = tuning_table()
    if args.tuning_table_out:
        adr.tuning_table_write(args.tuning_table_out)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one thread) ...")
        out["cpu_baseline"] = cpu_baseline(args, N, iters_d)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
