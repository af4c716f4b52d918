"""`cut_is_robust` (the guard of the kept-count comparisons) against the
oracle's own multiplet-safe truncation rule, by brute force on diagonal
environments whose spectra are moved by random perturbations."""

import json
import os

import numpy as np

from oracle import hotrg
from tests.sensitivity import cut_is_robust


def oracle_kept(spectrum, d_cut, tau):
    return hotrg.projector(np.diag(spectrum), d_cut, "multiplet", tau)[3]


def test_robust_cuts_survive_perturbations():
    rng = np.random.default_rng(11)
    n, d_cut, tau = 24, 11, 1e-6  # an odd cut falls inside a pair
    robust_seen = fragile_seen = 0
    for _ in range(400):
        # clustered spectra: pairs whose splitting is near tau
        base = np.sort(rng.uniform(0.01, 1.0, n // 2))[::-1]
        split = tau * rng.uniform(0.0, 3.0, n // 2)
        s = np.sort(np.concatenate([base, base - split]))[::-1]
        s = s / s[0]
        delta = tau * rng.uniform(0.01, 1.0)
        if cut_is_robust(s, n, d_cut, tau, delta):
            robust_seen += 1
            want = oracle_kept(s, d_cut, tau)
            for _ in range(20):
                moved = s + rng.uniform(-delta, delta, n) * 0.999
                moved[0] = 1.0
                assert oracle_kept(moved, d_cut, tau) == want
        else:
            fragile_seen += 1
    assert robust_seen > 50 and fragile_seen > 50


def test_gap_at_threshold_is_fragile():
    s = np.array([1.0, 0.5, 0.5 - 1.05e-6, 0.2, 0.1])
    assert not cut_is_robust(s, 5, 2, 1e-6, 1e-7)
    assert cut_is_robust(s, 5, 2, 1e-6, 1e-9)
    assert cut_is_robust(s, 2, 2, 1e-6, 1.0)  # nothing truncated


def test_stored_xy_batch_keeps_most_cuts_comparable():
    path = os.path.join(os.path.dirname(__file__), "golden", "xy_batch.json")
    from tests.sensitivity import spectra_tolerances

    runs = json.load(open(path))["runs"]
    total = compared = 0
    for r in runs:
        tol = spectra_tolerances(r["spectra_drift"])
        for a, b, ws, t in zip(r["steps"], r["kept_perturbed"], r["spectra"], tol):
            ok = a["kept"] == b and cut_is_robust(ws, a["dx"] * a["dx"], a["d_new"], r["tau"], t)
            total += 1
            if not ok:
                break
            compared += 1
    # the guard drops only the cuts that rounding can move
    assert compared > 0.5 * total, (compared, total)
