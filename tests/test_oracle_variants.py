"""Pins of the oracle's method variants: the two-sided isometry choice and
the finite-difference internal energy and specific heat."""

import math

import numpy as np
import pytest

from oracle import exact, hotrg, tensors, thermo

UNTRUNCATED = 10**9


def random_tensor(seed, dx, dy):
    return np.random.default_rng(seed).random((dx, dy, dx, dy)) + 0.1


def test_two_sided_equals_one_sided_for_symmetric_tensors():
    # the Ising and XY tensors are symmetric under left-right reflection: both
    # environments coincide, the tie keeps the left one, and the runs agree
    for T in (tensors.ising(0.44), tensors.xy(1.0, 2)):
        a = hotrg.run(T, 8, 12, trunc="multiplet", tau=1e-10)
        b = hotrg.run(T, 8, 12, trunc="multiplet", tau=1e-10, isometry="two")
        assert b.lnz_per_site == a.lnz_per_site
        assert all(s.side == 0 for s in b.steps)


def test_two_sided_is_reflection_invariant():
    # a left-right mirror of the whole lattice leaves Z unchanged; the
    # two-sided choice sees the same pair of environments, swapped, and makes
    # the same (mirrored) choice, so ln Z/N is the same; the one-sided choice
    # truncates a different environment and in general does not agree
    T = random_tensor(11, 3, 3)
    two = hotrg.run(T, 4, 8, isometry="two").lnz_per_site
    two_m = hotrg.run(hotrg.mirror(T), 4, 8, isometry="two").lnz_per_site
    one = hotrg.run(T, 4, 8).lnz_per_site
    one_m = hotrg.run(hotrg.mirror(T), 4, 8).lnz_per_site
    assert two == pytest.approx(two_m, rel=1e-13)
    assert abs(one - one_m) > 1e-9


def test_two_sided_picks_the_rank_deficient_side():
    # T[l,u,r,d] = a[l] B[u,r,d]: the left legs carry a rank-one factor, so the
    # left environment has rank one and truncation error 0 at any D_cut; the
    # mirrored tensor must take its projector from the right environment
    rng = np.random.default_rng(5)
    a = rng.random(3) + 0.1
    B = rng.random((3, 3, 3)) + 0.1
    T = np.einsum("l,urd->lurd", a, B)
    _, _, _, _, side = hotrg.directional_step(T, 2, isometry="two")
    _, _, _, _, side_m = hotrg.directional_step(hotrg.mirror(T), 2, isometry="two")
    assert (side, side_m) == (0, 1)


def test_two_sided_untruncated_is_exact():
    # with nothing cut either projector is an exact resolution of identity on the kept space
    T = random_tensor(3, 2, 2)
    a = hotrg.run(T, UNTRUNCATED, 3).lnz_per_site
    b = hotrg.run(T, UNTRUNCATED, 3, isometry="two").lnz_per_site
    assert b == pytest.approx(a, rel=1e-13)


@pytest.mark.parametrize("T", [1.5, 3.5])
def test_finite_difference_energy_and_specific_heat_match_onsager(T):
    # D = 16, 30 directional steps (2^15 x 2^15 sites): ln Z/N is within ~1e-10
    # of Onsager here, so the five-point differences with h = 1e-3 carry the
    # exact derivatives to ~1e-8 (energy) and ~1e-6 (specific heat)
    beta = 1.0 / T
    r = thermo.thermo(tensors.ising, beta, 1e-3, 16, 30)
    assert r["energy"] == pytest.approx(exact.onsager_energy(beta), rel=1e-7)
    assert r["cv"] == pytest.approx(exact.onsager_specific_heat(beta), rel=1e-5)
    assert r["lnz"] == pytest.approx(exact.onsager_integral(beta), rel=1e-9)
