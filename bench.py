"""Benchmark of the HOTRG coarse-graining path on one MI355X.

Workload: 2D Ising at T_c = 2/ln(1+sqrt 2), D_cut = 64, 30 directional
coarse-graining steps (2^15 x 2^15 sites), synthetic (closed-form Boltzmann
weights, no dataset).  One bench *step* is one whole run through the C ABI
(hotrg_run: initial tensor, 30 directional steps, periodic trace), inputs
built on the host inside the call, so `ms_per_step` is milliseconds per
30-step run (`ms_per_directional_step` divides it by 30).  `value` is
directional coarse-graining steps per second over the timed runs.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|fp32|bf16x3]
                    [--no-cpu-baseline] [--no-compare] [--no-batch] [--no-serve] [--no-cases]
                    [--kernel-probe]

Prints one JSON line.  The headline (`value`) uses --prec contractions
(FP64 by default, the precision of the paper's runs); `mixed_vs_fp64`
repeats the workload with FP32 and split-BF16 x3 contractions (the FP64
eigensolver and log-norm accumulation are unchanged; min(K, 5) runs each),
and with the precision chosen for a stated tolerance of 1e-7 (HOTRG_PREC_AUTO),
and states each result's ln Z/N error against the stored FP64 oracle.
`batch` runs the 64-problem XY batch; `serve` a seeded Poisson stream of 20
mixed requests (p50/p99 latency, each result's stated error bound);
`cpu_baseline` times the oracle on the host cores (one steady D = 64 step;
whole runs at D_cut = 32 and 8 on all cores and on one core).  The dominant kernel
is the D^7 contraction (C2); its average duration over the steady-state
steps of the timed runs comes from HIP events recorded on the library's
stream around each phase.

    python bench.py --batch             # 64 XY problems on the worker pool
    python bench.py --batch --batch-engine lockstep   # ... in lockstep (grouped launches)
    python bench.py --serve N [--serve-loads 0.8,0.5,1.0,1.2]

`--serve` replays a seeded stream of N mixed requests at Poisson arrival
rates given as fractions of the saturation rate measured closed-loop on a
prefix; the first load is the result, the others go to `load_sweep`.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HOTRG steps/s + TFLOP/s at D=64 (mixed vs FP64), ln Z/N error, p50/p99 latency"
BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
ONSAGER_TC = math.log(2.0) / 2.0 + 2.0 * 0.915965594177219015054603514932384110774 / math.pi
PEAKS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}  # TFLOP/s, dense MFMA, MI355X
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}
# HBM bytes of one dominant-kernel launch at the steady-state shape, from the
# FETCH_SIZE / WRITE_SIZE counter runs of `bench.py --kernel-probe` (scaled by
# the readings of a 1 GiB copy); the summary and commands are under profiles/.
# An entry is valid only for the kernel version it was measured on.
TRAFFIC = {("fp64", 64): 9.648e10, ("fp32", 64): 3.866e10, ("bf16x3", 64): 3.022e10}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--d-cut", type=int, default=64)
    ap.add_argument("--n-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP32 / split-BF16 runs of the same workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch sub-record")
    ap.add_argument("--no-serve", action="store_true", help="skip the serve sub-record")
    ap.add_argument("--no-cases", action="store_true",
                    help="skip the D_cut = 8 and D_cut = 32 sub-records (for profiling one workload)")
    ap.add_argument("--cpu-baseline-child", type=int, default=0, metavar="THREADS",
                    help=argparse.SUPPRESS)
    ap.add_argument("--batch", action="store_true",
                    help="the 64-problem XY batch workload instead of the single Ising run")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="serve a seeded Poisson stream of N mixed requests instead")
    ap.add_argument("--no-serve-check", dest="serve_check", action="store_false",
                    help="skip the FP64 re-run of the served requests")
    ap.add_argument("--serve-check-max", type=int, default=40,
                    help="FP64 re-run of the first N served requests (bounded time)")
    ap.add_argument("--serve-loads", default="0.8",
                    help="comma-separated arrival rates as fractions of the measured "
                         "saturation rate; the stream at the first one is the result, "
                         "the others are reported under load_sweep")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--batch-engine", choices=["pool", "lockstep"], default="pool",
                    help="with --batch: the worker pool (and one stream), or the lockstep engine")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="run one coarse contraction at the benchmark shape and a 1 GiB "
                         "calibration copy (for hardware-counter runs), then exit")
    return ap.parse_args()


def kernel_probe(args):
    """One launch of each coarse contraction at D = d_cut (the shape of a
    steady-state benchmark step) in --prec arithmetic on seeded inputs,
    preceded by a device copy of exactly 1 GiB whose counter readings
    calibrate FETCH_SIZE/WRITE_SIZE.  (With the tuner on, the candidates of
    each product shape run too: set HOTRG_AUTOTUNE=0 and force the tile.)"""
    import torch

    from paper_2306_00358_amd import Context, hotrg_coarse

    D = args.d_cut
    n = 1 << 27  # 2^27 doubles = 1 GiB
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    g = torch.Generator(device="cuda").manual_seed(0)
    T = torch.rand((D, D, D, D), dtype=torch.float64, device="cuda", generator=g)
    U = torch.rand((D, D, D), dtype=torch.float64, device="cuda", generator=g)
    Tt = torch.empty_like(T)
    with Context(0) as ctx:
        hotrg_coarse(ctx, T, U, Tt, prec=args.prec)
    torch.cuda.synchronize()
    print(json.dumps({"kernel_probe": {"d": D, "prec": args.prec, "copy_bytes": 8 * n}}),
          flush=True)


def xy_batch_problems(prec):
    """The XY batch: beta_i = 0.8 + 0.6 i/63 (inclusive grid), n_max = 3 + (i mod 4),
    D_cut = (24, 32, 40, 48)[(i div 4) mod 4], 25 directional steps,
    multiplet-safe truncation with tau = 1e-5 (cuts only at gaps that one
    rounding cannot move)."""
    from paper_2306_00358_amd import make_opts, model_params

    probs = []
    for i in range(64):
        beta = 0.8 + 0.6 * i / 63.0
        n_max = 3 + (i % 4)
        d_cut = (24, 32, 40, 48)[(i // 4) % 4]
        tau = 1e-5
        probs.append((model_params("xy", beta=beta, n_max=n_max),
                      make_opts(d_cut, 25, prec=prec, trunc="multiplet", degen_tol=tau)))
    return probs


def run_batch_bench(args):
    import torch

    from paper_2306_00358_amd import Context, hotrg_run_batch
    from paper_2306_00358_amd.flops import dims_schedule, step_flops

    prec = args.prec if args.prec != "fp64" else "fp32"
    probs = xy_batch_problems(prec)
    P = [p for p, _ in probs]
    O = [o for _, o in probs]
    flops = sum(sum(step_flops(*d)["total"] for d in dims_schedule(2 * p.n_max + 1, o.d_cut, o.n_steps))
                for p, o in probs)
    n_dir = sum(o.n_steps for o in O)
    config = {"workload": "64 XY problems, beta in [0.8,1.4], n_max 3..6, D_cut in "
                          "{24,32,40,48}, 25 directional steps, %s contractions" % prec}

    if args.batch_engine == "lockstep":
        from paper_2306_00358_amd import hotrg_run_grouped

        with Context(0) as ctx:
            hotrg_run_grouped(ctx, P, O)  # warm-up: tile choices, workspaces, graphs
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, st = hotrg_run_grouped(ctx, P, O)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            stats = ctx.group_stats()
        assert st == [0] * len(P), st
        print(json.dumps({
            "metric": METRIC + " [XY batch, lockstep]", "value": n_dir / dt, "unit": "steps/s",
            "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": DTYPE[prec], "data": "synthetic", "config": config,
            "tflops": flops / dt / 1e12, "graph": stats,
            "lnz_per_site": [r["lnz_per_site"] for r in res]}), flush=True)
        return

    def timed(workers):
        with Context(0) as ctx:
            ctx.set_workers(workers)
            hotrg_run_batch(ctx, P[:workers], O[:workers])  # warm-up: workspaces, kernels
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, st = hotrg_run_batch(ctx, P, O)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        assert st == [0] * len(P), st
        return dt, [r["lnz_per_site"] for r in res]

    t_pool, lnz_pool = timed(args.workers)
    t_seq, lnz_seq = timed(1)
    same = all(a == b for a, b in zip(lnz_pool, lnz_seq))
    out = {
        "metric": METRIC + " [XY batch]",
        "value": n_dir / t_pool,
        "unit": "steps/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_pool * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic",
        "config": dict(config, workers=args.workers),
        "tflops": flops / t_pool / 1e12,
        "sequential_steps_per_s": n_dir / t_seq,
        "speedup_vs_sequential": t_seq / t_pool,
        "batch_equals_sequential": same,
        "lnz_per_site": lnz_pool,
    }
    print(json.dumps(out), flush=True)


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(msg, file=sys.stderr, flush=True)


def serve_requests(n, seed=0, tol=0.0):
    """The serving mix: Ising (T uniform in [1.5, 3.5]) or XY (beta uniform in
    [0.6, 1.6], n_max = 4, multiplet tau 1e-5) with probability 1/2 each,
    D_cut uniform in {16, 32, 48, 64, 80}, 20-40 directional steps, FP32 or
    split-BF16 x3 contractions with the tolerance `tol` (0: none);
    generator PCG64 with the given seed."""
    import numpy as np

    from paper_2306_00358_amd import make_opts, model_params

    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        if rng.random() < 0.5:
            p = model_params("ising", beta=1.0 / rng.uniform(1.5, 3.5))
            trunc, tau = "plain", 1e-10
        else:
            p = model_params("xy", beta=rng.uniform(0.6, 1.6), n_max=4)
            trunc, tau = "multiplet", 1e-5
        o = make_opts(int(rng.choice([16, 32, 48, 64, 80])), int(rng.integers(20, 41)),
                      prec=str(rng.choice(["fp32", "bf16x3"])), trunc=trunc, degen_tol=tau,
                      tol=tol)
        reqs.append((p, o))
    return reqs


def serve_stream(ctx, reqs, rate, seed, tag):
    """Submit the requests at Poisson arrival times of the given rate (seeded)
    and wait for all of them.  Returns (results, wall seconds)."""
    import numpy as np
    import torch

    from paper_2306_00358_amd import Ticket

    arrivals = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=len(reqs)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for (p, o), ta in zip(reqs, arrivals):
        while time.perf_counter() - t0 < ta:
            time.sleep(0.0005)
        tickets.append(Ticket(ctx, p, o))
        log("%s request %d/%d submitted at %.2f s" % (tag, len(tickets), len(reqs), ta))
    vals = []
    for i, t in enumerate(tickets):
        vals.append(t.value())
        log("%s request %d/%d done, latency %.2f s" % (tag, i + 1, len(reqs),
                                                      vals[-1]["t_end"] - vals[-1]["t_submit"]))
    return vals, time.perf_counter() - t0


def stream_summary(reqs, vals, dt, flops):
    import numpy as np

    lat = np.array([v["t_end"] - v["t_submit"] for v in vals])
    wait = np.array([v["t_start"] - v["t_submit"] for v in vals])
    return {
        "steps_per_s": sum(o.n_steps for _, o in reqs) / dt,
        "tflops": sum(flops) / dt / 1e12,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "queue_wait_p50_s": float(np.percentile(wait, 50)),
        "queue_wait_p99_s": float(np.percentile(wait, 99)),
        "fp64_reruns": sum(1 for v, (_, o) in zip(vals, reqs) if v["prec_used"] != o.prec),
    }


def run_serve_bench(args):
    from paper_2306_00358_amd import Context, Ticket
    from paper_2306_00358_amd.flops import dims_schedule, step_flops

    reqs = serve_requests(args.serve, seed=0)
    loads = [float(x) for x in args.serve_loads.split(",") if x.strip()]
    if not loads or min(loads) <= 0.0:
        raise SystemExit("--serve-loads needs positive fractions of the saturation rate")

    def d0(p):
        return 2 if p.model == 0 else 2 * p.n_max + 1

    flops = [sum(step_flops(*d)["total"] for d in dims_schedule(d0(p), o.d_cut, o.n_steps))
             for p, o in reqs]
    with Context(0) as ctx:
        ctx.set_workers(args.workers)
        # closed loop on a prefix: the saturation rate in requests/s
        n_pre = max(4, min(len(reqs), 2 * args.workers))
        t0 = time.perf_counter()
        pre = [Ticket(ctx, p, o) for p, o in reqs[:n_pre]]
        for i, t in enumerate(pre):
            t.value()
            log("closed-loop request %d/%d done" % (i + 1, n_pre))
        sat = n_pre / (time.perf_counter() - t0)
        rate = loads[0] * sat
        vals, dt = serve_stream(ctx, reqs, rate, 1, "load %.2f" % loads[0])
        stats = ctx.sched_stats()
        k = min(len(reqs), args.serve_check_max) if args.serve_check else 0
        errors = serve_errors(ctx, reqs[:k], vals[:k]) if k else None
        sweep = []
        for j, load in enumerate(loads[1:]):
            v2, dt2 = serve_stream(ctx, reqs, load * sat, 2 + j, "load %.2f" % load)
            sweep.append(dict(load=load, arrival_rate_per_s=load * sat,
                              **stream_summary(reqs, v2, dt2, flops)))
    main = stream_summary(reqs, vals, dt, flops)
    out = {
        "metric": METRIC + " [serving]",
        "value": main["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1, "steps": len(reqs), "warmup": n_pre,
        "ms_per_step": dt / len(reqs) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32/bf16x3", "data": "synthetic",
        "config": {"workload": "seeded Poisson stream of %d Ising/XY requests, D_cut in "
                               "{16..80}, 20-40 steps" % len(reqs),
                   "workers": args.workers, "load": loads[0], "arrival_rate_per_s": rate,
                   "saturation_rate_per_s": sat},
        "tflops": main["tflops"],
        "latency_p50_s": main["latency_p50_s"],
        "latency_p99_s": main["latency_p99_s"],
        "queue_wait_p50_s": main["queue_wait_p50_s"],
        "queue_wait_p99_s": main["queue_wait_p99_s"],
        "admission": stats,
        "fp64_reruns": main["fp64_reruns"],
        "lnz_rel_error_vs_fp64": errors,
        "lnz_error_checked_requests": k,
    }
    if sweep:
        out["load_sweep"] = sweep
    print(json.dumps(out), flush=True)


def serve_errors(ctx, reqs, vals):
    """ln Z/N of served results against the same requests with FP64
    contractions (the FP64 path matches the oracle to 1e-12); run after the
    timed stream on the requests given.  Summarised per requested precision
    and model."""
    import numpy as np

    from paper_2306_00358_amd import HotrgError, Ticket, make_opts

    tickets = [Ticket(ctx, p, make_opts(o.d_cut, o.n_steps, prec="fp64", trunc=o.trunc,
                                        degen_tol=o.degen_tol)) for p, o in reqs]
    out = {}
    for i, ((p, o), v, t) in enumerate(zip(reqs, vals, tickets)):
        try:
            r = t.value()
        except HotrgError as e:
            log("fp64 check %d/%d failed: %s" % (i + 1, len(reqs), e))
            continue
        log("fp64 check %d/%d done" % (i + 1, len(reqs)))
        key = "%s/%s" % ({0: "fp64", 1: "fp32", 2: "bf16x3"}[o.prec],
                         {0: "ising", 1: "xy"}.get(p.model, "other"))
        e = abs(v["lnz_per_site"] - r["lnz_per_site"]) / abs(r["lnz_per_site"])
        out.setdefault(key, []).append((e, v["prec_used"] != o.prec))
    return {k: {"n": len(v), "fp64_reruns": sum(f for _, f in v),
                "max": max(e for e, _ in v), "median": float(np.median([e for e, _ in v]))}
            for k, v in sorted(out.items())}


def batch_record(args):
    """The 64-problem XY batch (FP32 contractions): in lockstep (grouped
    launches, one HIP graph per sweep; after one untimed batch that tunes the
    grouped tiles), on the worker pool (after a warm-up batch of the first
    problems) and one problem after another on one stream; each result of the
    lockstep run against the pool's."""
    import torch

    from paper_2306_00358_amd import Context, hotrg_run_batch, hotrg_run_grouped
    from paper_2306_00358_amd.flops import dims_schedule, step_flops

    probs = xy_batch_problems("fp32")
    P = [p for p, _ in probs]
    O = [o for _, o in probs]
    flops = sum(sum(step_flops(*d)["total"] for d in dims_schedule(2 * p.n_max + 1, o.d_cut,
                                                                      o.n_steps))
                for p, o in probs)
    n_dir = sum(o.n_steps for o in O)
    with Context(0) as ctx:
        hotrg_run_grouped(ctx, P, O)
        torch.cuda.synchronize()
        s0 = ctx.group_stats()
        t0 = time.perf_counter()
        res_g, st_g = hotrg_run_grouped(ctx, P, O)
        torch.cuda.synchronize()
        dt_g = time.perf_counter() - t0
        s1 = ctx.group_stats()
    log("batch, lockstep: %d problems in %.2f s" % (len(P), dt_g))
    with Context(0) as ctx:
        ctx.set_workers(args.workers)
        hotrg_run_batch(ctx, P[:args.workers], O[:args.workers])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_p, st_p = hotrg_run_batch(ctx, P, O)
        torch.cuda.synchronize()
        dt_p = time.perf_counter() - t0
    log("batch, worker pool: %d problems in %.2f s" % (len(P), dt_p))
    from paper_2306_00358_amd import hotrg_run

    with Context(0) as ctx:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p, o in zip(P, O):
            hotrg_run(ctx, p, o)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
    log("batch, one problem after another: %d problems in %.2f s" % (len(P), dt_s))
    diff = [abs(a["lnz_per_site"] - b["lnz_per_site"]) / abs(b["lnz_per_site"])
            for a, b in zip(res_g, res_p) if a and b]
    stats = {k: s1[k] - s0[k] for k in s1}
    return {"workload": "64 XY problems, beta in [0.8,1.4], n_max 3..6, D_cut in {24,32,40,48}, "
                        "25 directional steps, fp32 contractions, multiplet tau 1e-5",
            "engine": "lockstep: grouped launches, batched eigensolver, one HIP graph per sweep",
            "steps_per_s": n_dir / dt_g, "tflops": flops / dt_g / 1e12, "seconds": dt_g,
            "failed": sum(1 for x in st_g if x != 0), "graph": stats,
            "worker_pool": {"workers": args.workers, "steps_per_s": n_dir / dt_p,
                            "tflops": flops / dt_p / 1e12, "seconds": dt_p,
                            "failed": sum(1 for x in st_p if x != 0)},
            "sequential": {"steps_per_s": n_dir / dt_s, "tflops": flops / dt_s / 1e12,
                           "seconds": dt_s},
            "speedup_vs_worker_pool": dt_p / dt_g,
            "speedup_vs_sequential": dt_s / dt_g,
            "max_rel_diff_vs_worker_pool": max(diff) if diff else None,
            "max_stated_error_bound": max(r["err_bound"] for r in res_g if r)}


def serve_record(args, rate_tflops, n=20, tol=1e-7):
    """A seeded Poisson stream of n mixed requests (the serving mix, each
    with a stated tolerance of tol against FP64) at 0.8 of the saturation
    rate estimated from rate_tflops over the mean request's flops."""
    import numpy as np

    from paper_2306_00358_amd import Context
    from paper_2306_00358_amd.flops import dims_schedule, step_flops

    reqs = serve_requests(n, seed=0, tol=tol)

    def d0(p):
        return 2 if p.model == 0 else 2 * p.n_max + 1

    flops = [sum(step_flops(*d)["total"] for d in dims_schedule(d0(p), o.d_cut, o.n_steps))
             for p, o in reqs]
    sat = rate_tflops * 1e12 / float(np.mean(flops))
    rate = 0.8 * sat
    with Context(0) as ctx:
        ctx.set_workers(args.workers)
        vals, dt = serve_stream(ctx, reqs, rate, 1, "serve")
        stats = ctx.sched_stats()
    out = stream_summary(reqs, vals, dt, flops)
    bounds = {}
    for (p, o), v in zip(reqs, vals):
        key = "%s/%s" % ({0: "fp64", 1: "fp32", 2: "bf16x3"}[v["prec_used"]],
                         {0: "ising", 1: "xy"}.get(p.model, "other"))
        bounds.setdefault(key, []).append(v["err_bound"])
    out.update({
        "workload": "seeded Poisson stream of %d Ising/XY requests, D_cut in {16..80}, 20-40 "
                    "steps, fp32 / split-bf16 contractions with tol %.0e against FP64" % (n, tol),
        "arrival_rate_per_s": rate, "estimated_saturation_per_s": sat,
        "admission": stats, "seconds": dt,
        "stated_error_bound": {k: {"n": len(b), "max": max(b), "median": float(np.median(b))}
                               for k, b in sorted(bounds.items())},
    })
    return out


def small_case(ctx, reps=20):
    """The small configuration (Ising at T_c, D_cut = 8, 20 directional steps,
    FP64): launch- and latency-bound; steps/s over `reps` runs, step by step
    (hotrg_run) and with the steady steps replayed as one captured HIP graph
    per sweep (hotrg_run_grouped with one problem)."""
    import torch

    from paper_2306_00358_amd import hotrg_run, hotrg_run_grouped, make_opts, model_params

    params = model_params("ising", beta=BETA_C)
    opts = make_opts(8, 20)
    hotrg_run(ctx, params, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = hotrg_run(ctx, params, opts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    hotrg_run_grouped(ctx, [params], [opts])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = hotrg_run_grouped(ctx, [params], [opts])[0][0]
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t0) / reps
    return {"workload": "Ising T_c, D_cut=8, 20 directional steps, fp64", "steps_per_s": 20 / dt,
            "ms_per_run": dt * 1e3,
            "rel_err_vs_onsager": abs(r["lnz_per_site"] - ONSAGER_TC) / ONSAGER_TC,
            "graph": {"steps_per_s": 20 / dg, "ms_per_run": dg * 1e3,
                      "rel_diff_vs_step_by_step": abs(g["lnz_per_site"] - r["lnz_per_site"])
                      / abs(r["lnz_per_site"])}}


def mid_case(ctx, reps=3):
    """The D_cut = 32 configuration: Ising at T = 2.0, T_c and 2.5, 30
    directional steps, FP64; steps/s over `reps` runs per temperature."""
    import torch

    from paper_2306_00358_amd import hotrg_run, make_opts, model_params

    runs = []
    for T in (2.0, None, 2.5):
        beta = BETA_C if T is None else 1.0 / T
        params = model_params("ising", beta=beta)
        opts = make_opts(32, 30)
        hotrg_run(ctx, params, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = hotrg_run(ctx, params, opts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        runs.append({"T": 1.0 / beta, "steps_per_s": 30 / dt, "ms_per_run": dt * 1e3,
                     "lnz_per_site": r["lnz_per_site"]})
    return {"workload": "Ising at T = 2.0, T_c, 2.5; D_cut=32, 30 directional steps, fp64",
            "runs": runs}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_full_runs(threads):
    """The oracle's whole runs (initial tensor to ln Z / N) of the small and
    the D_cut = 32 configurations (Ising at T_c), with `threads` BLAS threads
    (0: all available)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import hotrg, tensors

    out = {}
    with threadpool_limits(threads if threads > 0 else None):
        used = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        for name, d_cut, K in (("d_cut_8", 8, 20), ("d_cut_32", 32, 30)):
            t0 = time.perf_counter()
            r = hotrg.run(tensors.ising(BETA_C), d_cut, K)
            dt = time.perf_counter() - t0
            out[name] = {"seconds": dt, "steps_per_s": K / dt, "threads": used,
                         "lnz_per_site": r.lnz_per_site,
                         "workload": "Ising T_c, D_cut=%d, %d directional steps, init to ln Z/N"
                                     % (d_cut, K)}
    return out


def cpu_baseline(d_cut):
    """The oracle on the host cores: one steady-state directional step at
    dims (d_cut, d_cut, d_cut) of the same Ising run (the warm-up steps that
    produce its input are not timed)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import hotrg, tensors

    T = tensors.ising(BETA_C)
    T = T / np.abs(T).max()
    k = 0
    while not (T.shape[0] == d_cut and T.shape[1] == d_cut):
        Tt = hotrg.directional_step(T, d_cut)[0]
        T = hotrg.rotate(Tt)
        T = T / np.abs(T).max()
        k += 1
        if k > 12:
            raise RuntimeError("steady state not reached")
    t0 = time.perf_counter()
    Tt = hotrg.directional_step(T, d_cut)[0]
    T = hotrg.rotate(Tt)
    T = T / np.abs(T).max()
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    from paper_2306_00358_amd.flops import step_flops

    f = step_flops(d_cut, d_cut, d_cut)["total"]
    return {"value": 1.0 / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": "one steady-state directional step (dims %d,%d,%d; step %d of the T_c run), "
                      "numpy/OpenBLAS FP64, %.1f s, %.3f TFLOP/s" % (d_cut, d_cut, d_cut, k + 1, dt,
                                                                     f / dt / 1e12)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    if args.cpu_baseline_child:
        # the oracle's whole runs on a fixed number of host threads (no GPU)
        print(json.dumps(cpu_full_runs(args.cpu_baseline_child)), flush=True)
        return
    child = None
    if not (args.no_cpu_baseline or args.kernel_probe or args.batch or args.serve):
        # the one-core oracle runs overlap the GPU measurements: a child
        # process started before this one touches the GPU
        import subprocess

        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
        child = subprocess.Popen([sys.executable, os.path.abspath(__file__),
                                  "--cpu-baseline-child", "1"], stdout=subprocess.PIPE,
                                 stderr=subprocess.DEVNULL, env=env, text=True)

    import torch

    from paper_2306_00358_amd import Context, hotrg_run, make_opts, model_params
    from paper_2306_00358_amd.flops import dims_schedule, step_flops

    assert torch.cuda.is_available(), "no GPU"
    if args.kernel_probe:
        kernel_probe(args)
        return
    if args.batch:
        run_batch_bench(args)
        return
    if args.serve:
        run_serve_bench(args)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = Context(0)
    params = model_params("ising", beta=BETA_C)
    sched = dims_schedule(2, args.d_cut, args.n_steps)
    flops_run = sum(step_flops(*d)["total"] for d in sched)
    steady = (args.d_cut, args.d_cut, args.d_cut)
    golden = os.path.join(ROOT, "tests", "golden", "ising_d64.json")
    ref = None
    if args.d_cut == 64 and args.n_steps <= 40 and os.path.exists(golden):
        with open(golden) as f:
            ref = json.load(f)["runs"][0]["steps"][args.n_steps - 1]["lnz_torus"]

    def measure(prec, runs=None, warmup=None, tol=0.0):
        runs = args.steps if runs is None else runs
        warmup = args.warmup if warmup is None else warmup
        opts = make_opts(args.d_cut, args.n_steps, prec=prec, spec_len=0, tol=tol)
        for _ in range(warmup):
            hotrg_run(ctx, params, opts)
        ctx.timings()  # discard
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [hotrg_run(ctx, params, opts) for _ in range(runs)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ctx.enable_timing(False)
        recs = ctx.timings()
        log("%s%s: %d runs in %.2f s" % (prec, " tol %.0e" % tol if tol else "", runs, elapsed))
        c2 = [r["ms"] for r in recs
              if r["phase"] == "c2" and (r["dx"], r["dy"], r["d_new"]) == steady]
        phase_ms = {}
        for r in recs:
            phase_ms[r["phase"]] = phase_ms.get(r["phase"], 0.0) + r["ms"] / runs
        c2_ms = sum(c2) / len(c2) if c2 else float("nan")
        achieved = step_flops(*steady)["c2"] / (c2_ms * 1e-3) / 1e12
        lnz = results[-1]["lnz_per_site"]
        tflops = flops_run * runs / elapsed / 1e12
        pu = {0: "fp64", 1: "fp32", 2: "bf16x3"}[results[-1]["prec_used"]]
        issued = 3.0 if pu == "bf16x3" else 1.0  # bf16 products per multiply-add
        return {
            "runs": runs,
            "prec_used": pu,
            "err_bound": results[-1]["err_bound"],
            "steps_per_s": args.n_steps * runs / elapsed,
            "ms_per_run": elapsed / runs * 1e3,
            "tflops": tflops,
            # whole run: issued MFMA flops over run time x peak (eigensolver included)
            "run_frac_of_peak": issued * tflops / PEAKS[pu],
            "eigh_share": phase_ms.get("eigh", 0.0) / (elapsed / runs * 1e3),
            "lnz_per_site": lnz,
            "rel_err_vs_fp64_oracle": abs(lnz - ref) / abs(ref) if ref is not None else None,
            "rel_err_vs_onsager": abs(lnz - ONSAGER_TC) / ONSAGER_TC,
            "phase_ms_per_run": phase_ms,
            "c2_ms": c2_ms, "c2_launches": len(c2), "c2_tflops": achieved,
        }

    head = measure(args.prec)
    peak = PEAKS[args.prec]
    out = {
        "metric": METRIC,
        "value": head["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_run"],
        "bench_step": "one whole run of %d directional steps" % args.n_steps,
        "ms_per_directional_step": head["ms_per_run"] / args.n_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": "2D Ising HOTRG at Tc, D_cut=%d, %d directional steps, %s contractions"
                               % (args.d_cut, args.n_steps, args.prec),
                   "d_cut": args.d_cut, "n_steps": args.n_steps, "prec": args.prec,
                   "beta": BETA_C},
        "tflops": head["tflops"],
        "lnz_per_site": head["lnz_per_site"],
        "rel_err_vs_onsager": head["rel_err_vs_onsager"],
        "rel_err_vs_oracle": head["rel_err_vs_fp64_oracle"],
        "phase_ms_per_run": head["phase_ms_per_run"],
        "roofline": {"bound": "mfma", "achieved": head["c2_tflops"], "peak": peak,
                     "unit": "TFLOP/s", "frac": head["c2_tflops"] / peak,
                     "traffic": TRAFFIC.get((args.prec, args.d_cut)),
                     "kernel": "C2 GEMM %dx%dx%d" % (args.d_cut**3, args.d_cut**2, args.d_cut**2),
                     "kernel_ms": head["c2_ms"], "launches": head["c2_launches"]},
    }
    out["run_frac_of_peak"] = head["run_frac_of_peak"]
    out["eigh_share"] = head["eigh_share"]
    if not args.no_cases:
        out["small_case"] = small_case(ctx)
        out["mid_case"] = mid_case(ctx)
    if not args.no_compare:
        # the same workload with reduced-precision contractions (eigensolver
        # and log-norm stay FP64)
        mixed = {}
        runs = min(args.steps, 5)
        for prec in ("fp32", "bf16x3"):
            if prec == args.prec:
                continue
            m = measure(prec, runs=runs, warmup=1)
            m["speedup_vs_" + args.prec] = m["steps_per_s"] / head["steps_per_s"]
            m["c2_frac_of_peak"] = m["c2_tflops"] / PEAKS[prec]
            # HBM bytes of one C2 launch (counters, profiles/), for this kernel version
            m["c2_traffic_bytes"] = TRAFFIC.get((prec, args.d_cut))
            if prec == "bf16x3":
                # three bf16 products are issued per multiply-add
                m["c2_issued_frac_of_peak"] = 3 * m["c2_tflops"] / PEAKS[prec]
            mixed[prec] = m
        # the cheapest precision whose stated bound meets 1e-7 (leading steps
        # FP64, the rest reduced)
        m = measure("auto", runs=runs, warmup=1, tol=1e-7)
        m["speedup_vs_" + args.prec] = m["steps_per_s"] / head["steps_per_s"]
        for k in ("c2_ms", "c2_launches", "c2_tflops"):
            m.pop(k)  # C2 launches of two precisions
        mixed["auto_tol_1e-7"] = m
        out["mixed_vs_" + args.prec] = mixed
    ctx.close()
    if not args.no_batch:
        out["batch"] = batch_record(args)
    if not args.no_serve:
        rate = (out.get("mixed_vs_" + args.prec, {}).get("auto_tol_1e-7", {}).get("tflops")
                or head["tflops"])
        out["serve"] = serve_record(args, rate)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.d_cut)
        cb["cpu_model"] = cpu_model()
        cb["full_runs_all_cores"] = cpu_full_runs(0)
        one = None
        if child is not None:
            try:
                one = json.loads(child.communicate(timeout=600)[0].strip().splitlines()[-1])
            except Exception as e:  # noqa: BLE001 - reported, not fatal
                child.kill()
                one = {"error": str(e)}
        cb["full_runs_one_core"] = one
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
