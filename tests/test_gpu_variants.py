"""Method variants on the GPU against the oracle: the generalized XY model,
the two-sided isometry choice and the finite-difference internal energy and
specific heat (hotrg_thermo)."""

import math
import sys

import numpy as np
import pytest

from oracle import exact, hotrg, tensors, thermo
from tests.inputs import random_tensor
from tests.sensitivity import oracle_drift, spectra_tolerances

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2306_00358_amd import Context

    c = Context(0)
    yield c
    c.close()


def test_gxy_matches_oracle(ctx):
    # multiplet tolerance 1e-5: every cut lies at a gap one rounding cannot
    # move, so the oracle is conditioned and the bar is the flat 1e-12
    from paper_2306_00358_amd import hotrg_run, make_opts, model_params

    beta, delta, n_max, D, K, tau = 1.0, 0.5, 3, 16, 12, 1e-5
    say("gxy beta", beta, "delta", delta, "n_max", n_max, "D", D, "K", K)
    got = hotrg_run(ctx, model_params("gxy", beta=beta, delta=delta, n_max=n_max),
                    make_opts(D, K, trunc="multiplet", degen_tol=tau, spec_len=D + 1))
    T0 = tensors.gxy(beta, delta, n_max)
    drift, lnz_drift, kept_pert, want = oracle_drift(T0, D, K, D + 1, trunc="multiplet", tau=tau)
    assert lnz_drift <= 1e-13 and kept_pert == [s.kept for s in want.steps]
    rel = abs(got["lnz_per_site"] - want.lnz_per_site) / abs(want.lnz_per_site)
    say("  rel", rel, "oracle drift", lnz_drift)
    assert rel <= 1e-12
    assert [a["kept"] for a in got["steps"]] == [b.kept for b in want.steps]
    tol = spectra_tolerances(drift)
    for k, (gs, ws) in enumerate(zip(got["spectra"], want.spectra)):
        n = min(len(gs), len(ws))
        assert np.abs(np.asarray(gs[:n]) - np.asarray(ws[:n])).max() <= tol[k], k


def test_gxy_at_delta_one_is_xy(ctx):
    from paper_2306_00358_amd import hotrg_run, make_opts, model_params

    o = make_opts(12, 10, trunc="multiplet", degen_tol=1e-10)
    a = hotrg_run(ctx, model_params("gxy", beta=1.1, delta=1.0, n_max=3), o)["lnz_per_site"]
    b = hotrg_run(ctx, model_params("xy", beta=1.1, n_max=3), o)["lnz_per_site"]
    assert a == b


def test_two_sided_matches_oracle_on_a_non_symmetric_tensor(ctx):
    from paper_2306_00358_amd import hotrg_run, make_opts, model_params

    T = random_tensor(3, 3, seed=21, positive=True)
    D, K = 6, 10
    say("two-sided raw 3x3, D", D, "K", K)
    got = hotrg_run(ctx, model_params("raw", raw=T), make_opts(D, K, isometry="two", spec_len=D + 1))
    want = hotrg.run(T, D, K, isometry="two", spec_len=D + 1)
    rel = abs(got["lnz_per_site"] - want.lnz_per_site) / abs(want.lnz_per_site)
    say("  rel", rel, "sides", [s["side"] for s in got["steps"]])
    assert rel <= 1e-12
    assert [s["side"] for s in got["steps"]] == [s.side for s in want.steps]
    assert any(s.side == 1 for s in want.steps)  # the case exercises both sides
    for g, w in zip(got["spectra"], want.spectra):
        n = min(len(g), len(w))
        assert np.abs(np.asarray(g[:n]) - w[:n]).max() <= 1e-12


def test_two_sided_keeps_one_sided_result_for_ising(ctx):
    from paper_2306_00358_amd import hotrg_run, make_opts, model_params

    p = model_params("ising", beta=0.44)
    a = hotrg_run(ctx, p, make_opts(16, 16))
    b = hotrg_run(ctx, p, make_opts(16, 16, isometry="two"))
    assert a["lnz_per_site"] == b["lnz_per_site"]
    assert all(s["side"] == 0 for s in b["steps"])


def test_two_sided_needs_fp64(ctx):
    from paper_2306_00358_amd import HotrgError, hotrg_run, make_opts, model_params
    from paper_2306_00358_amd._lib import HOTRG_ERR_INVALID

    with pytest.raises(HotrgError) as e:
        hotrg_run(ctx, model_params("ising", beta=0.44), make_opts(16, 8, prec="bf16x3",
                                                                   isometry="two"))
    assert e.value.status == HOTRG_ERR_INVALID


def test_thermo_matches_oracle_and_onsager(ctx):
    from paper_2306_00358_amd import hotrg_thermo, make_opts, model_params

    beta, h = 1.0 / 3.5, 1e-3
    say("thermo beta", beta, "h", h)
    got = hotrg_thermo(ctx, model_params("ising", beta=beta), make_opts(8, 20), h)
    want = thermo.thermo(tensors.ising, beta, h, 8, 20)
    say("  gpu", got, "oracle", want)
    assert got["lnz"] == pytest.approx(want["lnz"], rel=1e-12)
    # the differences amplify 1e-12 relative ln Z/N differences by 1/h and 1/h^2
    assert got["energy"] == pytest.approx(want["energy"], rel=1e-8)
    assert got["cv"] == pytest.approx(want["cv"], rel=1e-5)
    big = hotrg_thermo(ctx, model_params("ising", beta=beta), make_opts(16, 30), h)
    assert big["energy"] == pytest.approx(exact.onsager_energy(beta), rel=1e-7)
    assert big["cv"] == pytest.approx(exact.onsager_specific_heat(beta), rel=1e-5)


def test_thermo_rejects_bad_step(ctx):
    from paper_2306_00358_amd import HotrgError, hotrg_thermo, make_opts, model_params

    with pytest.raises(HotrgError):
        hotrg_thermo(ctx, model_params("ising", beta=0.001), make_opts(8, 4), 1e-3)
