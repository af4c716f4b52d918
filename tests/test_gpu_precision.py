"""Reduced-precision contractions (FP32 MFMA, split BF16 x3 with FP32
accumulation) against the FP64 oracle.

Element-wise bounds follow from the arithmetic.  For a contraction over K
terms with per-product relative error at most e_p and FP32 accumulation,
|computed - exact| <= (e_p + K 2^-24) sum_k |a_k b_k|; chained contractions
add their bounds (first order), with the oracle's contraction of |T| and |U|
as the scale.  e_p = 2^-24 for FP32 inputs; for split BF16 x = hi + lo +
O(2^-16 |x|) and the dropped lo*lo term give e_p = 3 * 2^-16.  Storing an
intermediate adds its rounding (2^-24 FP32, 2^-16 split BF16).
"""

import json
import math
import os
import sys

import numpy as np
import pytest

from oracle import exact, hotrg, tensors
from tests.inputs import random_projector, random_tensor

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U24, U16 = 2.0**-24, 2.0**-16
EP = {"fp32": U24, "bf16x3": 3 * U16}
STORE = {"fp32": U24, "bf16x3": U16}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2306_00358_amd import Context

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    c = Context(0)
    yield c
    c.close()


def _gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("dx,dy,dn", [(2, 2, 4), (5, 7, 9), (16, 16, 16), (24, 24, 24), (13, 40, 33)])
def test_coarse_reduced_bound(ctx, prec, dx, dy, dn):
    import torch

    from paper_2306_00358_amd import hotrg_coarse

    T = random_tensor(dx, dy, seed=400 + dx + dy)
    U = random_projector(dx, dn, seed=500 + dn)
    want = hotrg.coarse_tensor(T, U)
    scale = hotrg.coarse_tensor(np.abs(T), np.abs(U))
    Tt = torch.empty((dn, dy, dn, dy), dtype=torch.float64, device="cuda")
    hotrg_coarse(ctx, _gpu(T), _gpu(U), Tt, prec=prec)
    got = Tt.cpu().numpy()
    ks = [dx, dx * dy, dx * dx]
    # input rounding of T (twice) and U (twice) is inside e_p for split BF16;
    # for FP32 it adds 4 roundings
    bound = (3 * EP[prec] + sum(ks) * U24 + 2 * STORE[prec] + (4 * U24 if prec == "fp32" else 0))
    err = np.abs(got - want)
    say(prec, dx, dy, dn, "max err/scale %.3e bound %.3e rms rel %.3e" % (
        (err / scale).max(), bound, np.sqrt((err**2).mean()) / np.sqrt((want**2).mean())))
    assert np.all(err <= bound * scale)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("dx,dy", [(4, 16), (16, 16), (24, 24)])
def test_environment_reduced_bound(ctx, prec, dx, dy):
    import torch

    from paper_2306_00358_amd import hotrg_environment

    T = random_tensor(dx, dy, seed=600 + dx + dy)
    want = hotrg.environment(T)
    scale = hotrg.environment(np.abs(T))
    M = torch.empty((dx * dx, dx * dx), dtype=torch.float64, device="cuda")
    hotrg_environment(ctx, _gpu(T), M, prec=prec)
    got = M.cpu().numpy()
    P, K2 = dx * dy, dy * dy
    bound = 2 * EP[prec] + (P + K2) * U24 + STORE[prec] + (4 * U24 if prec == "fp32" else 0)
    err = np.abs(got - want)
    say(prec, dx, dy, "max err/scale %.3e bound %.3e" % ((err / scale).max(), bound))
    assert np.all(err <= bound * scale)


def _run(ctx, d_cut, K, prec, beta, spec_len=0):
    from paper_2306_00358_amd import hotrg_run, make_opts, model_params

    return hotrg_run(ctx, model_params("ising", beta=beta), make_opts(d_cut, K, prec=prec,
                                                                      spec_len=spec_len))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_run_dcut32_reduced_vs_fp64_oracle(ctx, prec):
    with open(os.path.join(GOLDEN, "ising_d32.json")) as f:
        runs = json.load(f)["runs"]
    for rec in runs:
        got = _run(ctx, 32, 30, prec, rec["beta"])
        rel = abs(got["lnz_per_site"] - rec["lnz_per_site"]) / abs(rec["lnz_per_site"])
        say(prec, "D=32 beta %.6f lnZ/N %.15f oracle %.15f rel %.3e" % (
            rec["beta"], got["lnz_per_site"], rec["lnz_per_site"], rel))
        # the steps before the steady state run in FP64; the stated target
        # of the reduced paths is 1e-7 relative
        assert rel <= 1e-7


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_run_dcut64_reduced_vs_fp64_oracle(ctx, prec):
    with open(os.path.join(GOLDEN, "ising_d64.json")) as f:
        rec = json.load(f)["runs"][0]
    got = _run(ctx, 64, 30, prec, rec["beta"])
    ref = rec["steps"][29]["lnz_torus"]
    rel = abs(got["lnz_per_site"] - ref) / abs(ref)
    say(prec, "D=64 K=30 lnZ/N %.15f oracle %.15f rel %.3e onsager rel %.3e" % (
        got["lnz_per_site"], ref, rel, abs(got["lnz_per_site"] - exact.onsager_tc()) / exact.onsager_tc()))
    assert rel <= 1e-7


@pytest.mark.parametrize("prec, u", [("fp64", 0.0), ("fp32", 2.0 ** -24), ("bf16x3", 2.0 ** -17)])
def test_eigensolver_residual_matches_the_step_precision(ctx, prec, u):
    # the last step of a D_cut = 32 run at T_c (n = 1024: the block solver)
    # stops at a relative Ritz residual of 5e-14 when it is FP64 and of
    # 2^-10 u_p when its contractions ran in precision p, whose environment
    # already carries rounding of relative size u_p
    beta = math.log(1.0 + math.sqrt(2.0)) / 2.0
    got = _run(ctx, 32, 30, prec, beta)
    sweeps, resid = ctx.last_eig()
    tol = max(5e-14, u * 2.0 ** -10)
    say(prec, "last solve: sweeps", sweeps, "residual %.3e" % resid, "target %.3e" % tol,
        "lnZ/N %.15f" % got["lnz_per_site"])
    assert sweeps > 0
    assert resid <= tol
