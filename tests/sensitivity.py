"""Conditioning of the oracle's per-step spectra, used to set the spectra
tolerance of the parity tests.

The spectra after step k depend on every earlier truncation.  Where the RG
flow amplifies perturbations (at T_c, the thermal direction is relevant) or a
cut falls at a noise-level gap (ordered phase), two correct FP64
implementations drift apart by far more than one rounding error.  This
module measures the drift of the oracle against itself when the environment
M of every step is perturbed by a seeded symmetric random matrix of relative
size 2^-52 (one rounding error); the parity tolerance of step k is then
max(floor, factor * drift_k).  The same perturbed run gives the drift of
ln Z/N and the kept counts a perturbed but correct run may choose; the
ln Z/N tolerance is max(floor, factor * lnz drift), and kept counts are
compared only at steps where the perturbed run kept the same number.
"""

import numpy as np

from oracle import hotrg

SPEC_FLOOR = 1e-12
SPEC_FACTOR = 100.0


LNZ_FLOOR = 1e-12
LNZ_FACTOR = 100.0


def oracle_drift(T0, d_cut, n_steps, spec_len, trunc="plain", tau=1e-10, seed=0, base=None):
    """Plain oracle run against one with every environment perturbed.
    Returns (per-step spectra drift, relative ln Z/N drift, perturbed kept
    counts, plain Result)."""
    rng = np.random.default_rng(seed)
    plain = base if base is not None else hotrg.run(T0, d_cut, n_steps, trunc, tau, spec_len)
    orig = hotrg.projector

    def perturbed(M, dc, tr="plain", ta=1e-10):
        E = rng.standard_normal(M.shape) * (2.0**-52) * np.abs(M).max()
        return orig(M + 0.5 * (E + E.T), dc, tr, ta)

    hotrg.projector = perturbed
    try:
        pert = hotrg.run(T0, d_cut, n_steps, trunc, tau, spec_len)
    finally:
        hotrg.projector = orig
    drift = []
    for a, b in zip(plain.spectra, pert.spectra):
        n = min(len(a), len(b))
        drift.append(float(np.abs(a[:n] - b[:n]).max()))
    lnz = abs(pert.lnz_per_site - plain.lnz_per_site) / abs(plain.lnz_per_site)
    return drift, float(lnz), [s.kept for s in pert.steps], plain


def spectra_drift(T0, d_cut, n_steps, spec_len, trunc="plain", tau=1e-10, seed=0, base=None):
    """Per-step max |spectrum difference| between the plain oracle run and
    the perturbed one.  Returns (drift list, plain Result)."""
    drift, _, _, plain = oracle_drift(T0, d_cut, n_steps, spec_len, trunc, tau, seed, base)
    return drift, plain


def spectra_tolerances(drift):
    return [max(SPEC_FLOOR, SPEC_FACTOR * d) for d in drift]


def lnz_tolerance(lnz_drift):
    return max(LNZ_FLOOR, LNZ_FACTOR * lnz_drift)
