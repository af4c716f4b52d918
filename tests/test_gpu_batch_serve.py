"""Many problems on one GPU: batch runs and the serving loop.

Each problem's result must be the same alone and in the mix (same kernels,
same tile choices, fixed-order reductions: equal to the last bit), and
match the FP64 oracle; admission must respect the HBM budget; cancellation
and over-budget requests must fail cleanly.
"""

import json
import math
import os
import subprocess
import sys
import time

import numpy as np
import pytest

from oracle import hotrg, tensors
from tests.inputs import poisson_arrivals, serving_stream

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch


def _mix():
    from paper_2306_00358_amd import make_opts, model_params

    probs = []
    for i, (model, beta, dc, K, prec) in enumerate([
            ("ising", 0.44068679350977147, 16, 20, "fp64"),
            ("ising", 0.40, 24, 16, "fp32"),
            ("xy", 1.0, 24, 12, "fp64"),
            ("xy", 1.1, 16, 14, "bf16x3"),
            ("ising", 0.50, 32, 12, "fp64"),
            ("xy", 0.9, 32, 10, "fp32"),
            ("ising", 0.46, 8, 24, "bf16x3"),
            ("potts", math.log(1 + math.sqrt(3)), 12, 14, "fp64")]):
        kw = {"beta": beta}
        if model == "xy":
            kw["n_max"] = 2 + i % 3
        if model == "potts":
            kw["q"] = 3
        trunc = "multiplet" if model == "xy" else "plain"
        tau = 1e-5
        probs.append((model_params(model, **kw), make_opts(dc, K, prec=prec, trunc=trunc,
                                                           degen_tol=tau, spec_len=4)))
    return probs


def test_batch_equals_alone(torch_cuda):
    from paper_2306_00358_amd import Context, hotrg_run, hotrg_run_batch

    probs = _mix()
    # the mix runs first, so the GEMM tuner measures its candidates while
    # other problems load the GPU; the alone runs then reuse those choices
    with Context(0) as ctx:
        ctx.set_workers(4)
        got, st = hotrg_run_batch(ctx, [p for p, _ in probs], [o for _, o in probs], with_steps=True)
        stats = ctx.sched_stats()
    with Context(0) as solo:
        alone = [hotrg_run(solo, p, o) for p, o in probs]
    assert st == [0] * len(probs)
    for a, g in zip(alone, got):
        assert g["lnz_per_site"] == a["lnz_per_site"]
        assert np.array_equal(g["spectra"], a["spectra"])
    assert stats["admitted"] == len(probs)
    # alone in a fresh process, whose tuner measured without the mix: the
    # tiles may differ, so equal within the stated tolerance instead of
    # bitwise -- FP64 1e-12; reduced precision twice the result's stated
    # bound against FP64 (each run is within err_bound of the FP64 result)
    r = subprocess.run([sys.executable, "-m", "tests.alone_child"], cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    fresh = json.loads(r.stdout.strip().splitlines()[-1])
    for (p, o), g, f in zip(probs, got, fresh):
        rel = abs(g["lnz_per_site"] - f) / abs(f)
        say("fresh process", p.model, o.prec, "rel", rel)
        assert rel <= (1e-12 if o.prec == 0 else 2.0 * g["err_bound"])
    say("batch ok", stats)


def test_batch_fp64_vs_oracle(torch_cuda):
    from paper_2306_00358_amd import Context, hotrg_run_batch

    probs = [p for p in _mix() if p[1].prec == 0]
    with Context(0) as ctx:
        got, st = hotrg_run_batch(ctx, [p for p, _ in probs], [o for _, o in probs])
    assert st == [0] * len(probs)
    for (p, o), g in zip(probs, got):
        if p.model == 0:
            T0 = tensors.ising(p.beta)
        elif p.model == 1:
            T0 = tensors.xy(p.beta, p.n_max)
        else:
            T0 = tensors.potts(p.beta, p.q)
        want = hotrg.run(T0, o.d_cut, o.n_steps, "multiplet" if o.trunc else "plain", o.degen_tol)
        rel = abs(g["lnz_per_site"] - want.lnz_per_site) / abs(want.lnz_per_site)
        say("model", p.model, "d_cut", o.d_cut, "rel", rel)
        assert rel <= 1e-12


def _xy_golden():
    path = os.path.join(GOLDEN, "xy_batch.json")
    with open(path) as f:
        return json.load(f)["runs"]


def _xy_problems(runs, **kw):
    from paper_2306_00358_amd import make_opts, model_params

    params = [model_params("xy", beta=r["beta"], n_max=r["n_max"]) for r in runs]
    opts = [make_opts(r["d_cut"], r["n_steps"], trunc="multiplet", degen_tol=r["tau"],
                      spec_len=r["d_cut"] + 1, **kw) for r in runs]
    return params, opts


def _check_xy_fp64(runs, got, tag):
    # every stored run is conditioned (R19): ln Z/N at the flat 1e-12, kept counts
    # at every step, spectra at every step within the per-step tolerance
    from tests.sensitivity import spectra_tolerances

    assert all(r["conditioned"] for r in runs), [r["index"] for r in runs if not r["conditioned"]]
    worst = 0.0
    for r, g in zip(runs, got):
        rel = abs(g["lnz_per_site"] - r["lnz_per_site"]) / abs(r["lnz_per_site"])
        worst = max(worst, rel)
        assert rel <= 1e-12, (tag, r["index"], rel)
        assert [a["kept"] for a in g["steps"]] == [b["kept"] for b in r["steps"]], (tag, r["index"])
        tol = spectra_tolerances(r["spectra_drift"])
        for k, (gs, ws) in enumerate(zip(g["spectra"], r["spectra"])):
            n = min(len(gs), len(ws))
            assert np.abs(np.asarray(gs[:n]) - np.asarray(ws[:n])).max() <= tol[k], (tag, r["index"], k)
    say(tag, "worst ln Z/N rel", worst)


def test_xy_batch_vs_stored_oracle(torch_cuda):
    # the 64-problem XY batch (D_cut 24..48) in FP64 on the worker pool
    from paper_2306_00358_amd import Context, hotrg_run_batch

    runs = _xy_golden()
    assert len(runs) == 64
    params, opts = _xy_problems(runs)
    with Context(0) as ctx:
        got, st = hotrg_run_batch(ctx, params, opts, with_steps=True)
    assert st == [0] * len(runs)
    _check_xy_fp64(runs, got, "pool")


def test_xy_batch_lockstep_vs_stored_oracle(torch_cuda):
    # the same batch in lockstep (grouped launches, batched eigensolver, graphs)
    from paper_2306_00358_amd import Context, hotrg_run_grouped

    runs = _xy_golden()
    params, opts = _xy_problems(runs)
    with Context(0) as ctx:
        got, st = hotrg_run_grouped(ctx, params, opts, with_steps=True)
        stats = ctx.group_stats()
    say("group stats", stats)
    assert st == [0] * len(runs)
    assert stats["replays"] >= 20
    _check_xy_fp64(runs, got, "lockstep")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_xy_batch_reduced_precision_within_stated_bound(torch_cuda, prec):
    # reduced-precision contractions with a stated tolerance of 1e-7 against
    # FP64: every result within its own a-priori bound of the stored FP64 oracle
    # value, and every bound within the tolerance; then the batch workload as
    # specified (every steady step reduced), against its bound as well
    from paper_2306_00358_amd import Context, hotrg_run_grouped

    runs = _xy_golden()
    for tol in (1e-7, 0.0):
        params, opts = _xy_problems(runs, prec=prec, tol=tol)
        with Context(0) as ctx:
            got, st = hotrg_run_grouped(ctx, params, opts)
        assert st == [0] * len(runs)
        worst = 0.0
        for r, g in zip(runs, got):
            rel = abs(g["lnz_per_site"] - r["lnz_per_site"]) / abs(r["lnz_per_site"])
            worst = max(worst, rel / g["err_bound"])
            assert rel <= g["err_bound"], (prec, tol, r["index"], rel, g["err_bound"])
            if tol:
                assert g["err_bound"] <= tol
        say(prec, "tol", tol, "largest error / stated bound", worst)


def test_serving_stream_budget_cancel(torch_cuda):
    from paper_2306_00358_amd import (Context, HotrgError, Ticket, hotrg_footprint, hotrg_run,
                                      make_opts, model_params)
    from paper_2306_00358_amd._lib import HOTRG_ERR_CANCELLED, HOTRG_ERR_OOM, HOTRG_OK

    rng = np.random.default_rng(5)
    reqs = []
    for i in range(16):
        if rng.random() < 0.5:
            p = model_params("ising", beta=1.0 / rng.uniform(1.5, 3.5))
            trunc, tau = "plain", 1e-10
        else:
            p = model_params("xy", beta=rng.uniform(0.6, 1.6), n_max=2)
            trunc, tau = "multiplet", 1e-6
        o = make_opts(int(rng.choice([8, 16, 24])), int(rng.integers(8, 16)),
                      prec=str(rng.choice(["fp32", "bf16x3"])), trunc=trunc, degen_tol=tau)
        reqs.append((p, o))
    fps = [hotrg_footprint(p, o) for p, o in reqs]
    budget = int(2.5 * max(fps))
    arrivals = poisson_arrivals(len(reqs), rate=40.0, seed=6)
    with Context(0) as solo:
        alone = [hotrg_run(solo, p, o)["lnz_per_site"] for p, o in reqs]
    with Context(0, hbm_budget=budget) as ctx:
        ctx.set_workers(4)
        t0 = time.perf_counter()
        tickets = []
        for (p, o), ta in zip(reqs, arrivals):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.001)
            tickets.append(Ticket(ctx, p, o))
        # a request larger than the budget is refused at submission
        big = make_opts(64, 30)
        with pytest.raises(HotrgError) as e:
            Ticket(ctx, model_params("ising", beta=0.44), big)
        assert e.value.status == HOTRG_ERR_OOM
        # cancel one request (queued or running): it ends CANCELLED or OK
        victim = Ticket(ctx, model_params("ising", beta=0.44), make_opts(24, 40, prec="fp32"))
        victim.cancel()
        assert victim.wait() in (HOTRG_ERR_CANCELLED, HOTRG_OK)
        vals = [t.value() for t in tickets]
        stats = ctx.sched_stats()
    for v, a in zip(vals, alone):
        assert v["lnz_per_site"] == a
        assert v["t_submit"] <= v["t_start"] <= v["t_end"]
    assert stats["peak_reserved"] <= budget
    lat = sorted(v["t_end"] - v["t_submit"] for v in vals)
    say("serving ok", stats, "p50 %.3f s p99 %.3f s" % (lat[len(lat) // 2], lat[-1]))


def _oracle_request(req):
    model, beta, n_max, q, d_cut, n_steps = req
    T0 = {"ising": lambda: tensors.ising(beta), "xy": lambda: tensors.xy(beta, n_max),
          "potts": lambda: tensors.potts(beta, q)}[model]()
    trunc = "multiplet" if model == "xy" else "plain"
    return hotrg.run(T0, d_cut, n_steps, trunc, SERVE_TAU).lnz_per_site


SERVE_TAU = 1e-5  # multiplet tolerance of the XY requests


def test_served_fp64_stream_matches_oracle(torch_cuda):
    # a seeded Poisson stream through submit / wait on four workers; every
    # served FP64 result against the oracle at 1e-12 (the workload is pinned
    # as conditioned by tests/test_serving_workload.py)
    from paper_2306_00358_amd import Context, Ticket, make_opts, model_params

    reqs = serving_stream(12, seed=21)
    want = [_oracle_request(r) for r in reqs]
    arrivals = poisson_arrivals(len(reqs), rate=20.0, seed=22)
    with Context(0) as ctx:
        ctx.set_workers(4)
        t0 = time.perf_counter()
        tickets = []
        for (model, beta, n_max, q, d_cut, n_steps), ta in zip(reqs, arrivals):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.001)
            trunc = "multiplet" if model == "xy" else "plain"
            tickets.append(Ticket(ctx, model_params(model, beta=beta, n_max=n_max, q=q),
                                  make_opts(d_cut, n_steps, trunc=trunc, degen_tol=SERVE_TAU)))
        got = [t.value() for t in tickets]
        stats = ctx.sched_stats()
    for r, g, w in zip(reqs, got, want):
        rel = abs(g["lnz_per_site"] - w) / abs(w)
        say("served", r, "rel", rel)
        assert g["prec_used"] == 0
        assert rel <= 1e-12, (r, rel)
    assert stats["admitted"] == len(reqs)


def test_footprint_bounds_held_memory(torch_cuda):
    from paper_2306_00358_amd import Context, hotrg_footprint, hotrg_run, make_opts, model_params

    for p, o in [(model_params("ising", beta=0.44), make_opts(32, 12)),
                 (model_params("ising", beta=0.44), make_opts(32, 12, prec="bf16x3")),
                 (model_params("xy", beta=1.0, n_max=3), make_opts(24, 8, prec="fp32"))]:
        with Context(0) as ctx:
            hotrg_run(ctx, p, o)
            held = ctx.bytes_in_use()
        fp = hotrg_footprint(p, o)
        say("held", held, "footprint", fp)
        assert held <= fp


def test_numeric_failure_reruns_in_fp64(torch_cuda):
    # XY deep in the low-temperature phase: split-BF16 rounding breaks the
    # charge structure and the flow runs off (a non-positive final trace);
    # the serving loop re-runs such a request once in FP64.  Whichever way
    # this request ends, its value must be the FP64 one or close to it.
    from paper_2306_00358_amd import (HOTRG_BF16X3, HOTRG_FP64, Context, Ticket, hotrg_run,
                                      make_opts, model_params)

    p = model_params("xy", beta=1.1541, n_max=4)
    o = make_opts(32, 36, prec="bf16x3", trunc="multiplet", degen_tol=1e-5)
    o64 = make_opts(32, 36, prec="fp64", trunc="multiplet", degen_tol=1e-5)
    with Context(0) as ctx:
        ctx.set_workers(2)
        got = Ticket(ctx, p, o).value()
        want = hotrg_run(ctx, p, o64)["lnz_per_site"]
    say("prec_used", got["prec_used"], got["lnz_per_site"], want)
    assert math.isfinite(got["lnz_per_site"])
    if got["prec_used"] == HOTRG_FP64:
        assert got["lnz_per_site"] == want
    else:
        # within the result's own stated bound against FP64
        assert got["prec_used"] == HOTRG_BF16X3
        assert abs(got["lnz_per_site"] - want) <= got["err_bound"] * abs(want)


def test_released_ticket_is_forgotten(torch_cuda):
    from paper_2306_00358_amd import Context, Ticket, make_opts, model_params
    from paper_2306_00358_amd._lib import HOTRG_ERR_INVALID, HOTRG_OK

    with Context(0) as ctx:
        t = Ticket(ctx, model_params("ising", beta=0.44), make_opts(8, 10))
        assert t.wait() == HOTRG_OK
        assert t.poll() == HOTRG_OK  # still known after wait
        t.release()
        assert t.poll() == HOTRG_ERR_INVALID
        v = Ticket(ctx, model_params("ising", beta=0.44), make_opts(8, 10)).value()
        assert math.isfinite(v["lnz_per_site"])
