"""Conditioning of the oracle's per-step spectra, used to set the spectra
tolerance of the parity tests.

The spectra after step k depend on every earlier truncation.  Where the RG
flow amplifies perturbations (at T_c, the thermal direction is relevant) or a
cut falls at a noise-level gap (ordered phase), two correct FP64
implementations drift apart by far more than one rounding error.  This
module measures the drift of the oracle against itself when the environment
M of every step is perturbed by a seeded symmetric random matrix of relative
size 2^-52 (one rounding error); the spectra tolerance of step k is then
max(floor, factor * drift_k).  The same perturbed run gives the drift of
ln Z/N and the kept counts a perturbed but correct run chooses: a parity case
is *conditioned* when the kept counts do not move, ln Z/N moves far below the
1e-12 bar, and every gap the multiplet rule looks at clears the threshold by
more than the spectra can move (`cut_is_robust`: the rule is a step function
of the spectrum, so at a gap within that distance of tau both cuts would be
correct results).  Only conditioned cases are held to 1e-12 on ln Z/N.
"""

import numpy as np

from oracle import hotrg

SPEC_FLOOR = 1e-12
SPEC_FACTOR = 100.0


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


def cut_is_robust(spectrum, n, d_new, tau, delta):
    """Whether the multiplet-safe cut of a spectrum (lambda / lambda_1,
    descending, at least d_new + 1 values when d_new < n) stays the same
    when every value moves by at most ``delta``.  The rule lowers the kept
    count from d_new while the gap below it is at most tau; each gap it
    examines, the last one included, must differ from tau by more than
    2 * delta (a gap is the difference of two moved values)."""
    if d_new >= n:
        return True  # nothing is truncated
    s = np.asarray(spectrum, dtype=np.float64)
    kept = d_new
    while kept > 0:
        gap = s[kept - 1] - s[kept]
        if abs(gap - tau) <= 2.0 * delta:
            return False
        if gap > tau:
            return True
        kept -= 1
    return True
