"""The serving parity stream is conditioned (CPU, oracle only): for every
request, a one-rounding perturbation of each step's environment keeps the
kept counts and moves ln Z/N by at most 1e-13 (ten times below the bar), so the GPU's served FP64
results can be held to 1e-12 (tests/test_gpu_batch_serve.py)."""

import pytest

from oracle import tensors
from tests.inputs import serving_stream
from tests.sensitivity import oracle_drift

SERVE_TAU = 1e-5


@pytest.mark.slow
def test_serving_parity_stream_is_conditioned():
    for model, beta, n_max, q, d_cut, n_steps in serving_stream(12, seed=21):
        T0 = {"ising": lambda: tensors.ising(beta), "xy": lambda: tensors.xy(beta, n_max),
              "potts": lambda: tensors.potts(beta, q)}[model]()
        trunc = "multiplet" if model == "xy" else "plain"
        _, lnz_drift, kept_pert, base = oracle_drift(T0, d_cut, n_steps, 4, trunc=trunc,
                                                      tau=SERVE_TAU)
        assert [s.kept for s in base.steps] == kept_pert
        assert lnz_drift <= 1e-13, (model, beta, d_cut, lnz_drift)
