"""Pins of the exact reference values (closed forms and brute force) that the
oracle is checked against."""

import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.special import iv

from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("T", [1.5, 2.0, exact.TC_ISING, 2.5, 3.5])
def test_onsager_forms_agree(T):
    # the paper's 4F3 form (Sec. 3.2) against Onsager's integral form
    a = exact.onsager_hyper(1.0 / T)
    b = exact.onsager_integral(1.0 / T)
    assert a == pytest.approx(b, rel=2e-15 if T != exact.TC_ISING else 1e-14)


def test_onsager_at_tc_closed_form():
    bc = math.log(1 + math.sqrt(2)) / 2
    assert exact.onsager_hyper(bc, dps=40) == pytest.approx(exact.onsager_tc(), rel=1e-15)
    assert exact.onsager_tc() == pytest.approx(0.9296953983416102, rel=1e-15)


def test_tc_matches_paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        pv = json.load(f)
    assert exact.TC_ISING == pytest.approx(pv["ising"]["tc_approx"]["value"], abs=5e-4)


def _ising_enumerate(beta, Lx, Ly):
    # direct sum over all 2^(Lx*Ly) spin configurations
    Z = 0.0
    for spins in itertools.product([1, -1], repeat=Lx * Ly):
        s = np.array(spins).reshape(Ly, Lx)
        E = 0
        for y in range(Ly):
            for x in range(Lx):
                E += s[y, x] * s[y, (x + 1) % Lx] + s[y, x] * s[(y + 1) % Ly, x]
        Z += math.exp(beta * E)
    return math.log(Z) / (Lx * Ly)


@pytest.mark.parametrize("Lx,Ly", [(1, 1), (1, 2), (2, 2), (3, 2), (2, 4), (4, 4)])
def test_ising_transfer_matrix_vs_enumeration(Lx, Ly):
    beta = 0.41
    assert exact.ising_torus(beta, Lx, Ly) == pytest.approx(_ising_enumerate(beta, Lx, Ly), rel=1e-14)


def test_ising_torus_large_lattice_tends_to_onsager():
    # deep in the disordered phase (T = 10) finite-size effects decay like
    # exp(-L/xi) with xi < 1: a 10x10 torus is within 1e-9 of the infinite lattice
    beta = 1.0 / 10.0
    assert exact.ising_torus(beta, 10, 10) == pytest.approx(exact.onsager_hyper(beta), rel=1e-9)


@pytest.mark.parametrize("beta", [0.3, 0.9])
def test_xy_torus_closed_forms(beta):
    # 1x1: Z = e^(2 beta); 1x2: Z = e^(2 beta) I0(2 beta) (two bonds between the sites)
    assert exact.xy_torus(beta, 1, 1) == pytest.approx(2 * beta, rel=1e-14)
    want = (2 * beta + math.log(iv(0, 2 * beta))) / 2
    assert exact.xy_torus(beta, 1, 2) == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("beta", [0.2, 1.0 / 1.5, 0.3, 1.0 / 3.5])
def test_onsager_energy_is_derivative_of_free_energy(beta):
    # closed form (elliptic K) against mpmath's derivative of the 4F3 form
    import mpmath as mp

    with mp.workdps(40):
        def f(b):
            kap = mp.sinh(2 * b) / (2 * mp.cosh(2 * b) ** 2)
            F = mp.hyper([1, 1, mp.mpf(3) / 2, mp.mpf(3) / 2], [2, 2, 2], 16 * kap**2)
            return mp.log(2 * mp.cosh(2 * b)) - kap**2 * F

        want = float(-mp.diff(f, mp.mpf(beta)))
    assert exact.onsager_energy(beta) == pytest.approx(want, rel=1e-13)


def test_onsager_energy_and_specific_heat_limits():
    # high temperature: ln Z/N = ln 2 + 2 ln cosh(beta) + O(beta^4 tanh^4) -> u ~ -2 tanh(beta)
    b = 1e-3
    assert exact.onsager_energy(b) == pytest.approx(-2 * math.tanh(b), rel=1e-5)
    assert exact.onsager_specific_heat(b) == pytest.approx(2 * b * b, rel=1e-4)
    # ground state: u -> -2 J per site
    assert exact.onsager_energy(5.0) == pytest.approx(-2.0, abs=1e-12)
