"""Pins of the oracle's initial tensors against closed forms."""

import math

import numpy as np
import pytest
from scipy.special import iv

from oracle import tensors


@pytest.mark.parametrize("beta", [0.1, 0.3, math.log(1 + math.sqrt(2)) / 2, 0.7])
def test_ising_closed_form(beta):
    # T[i,j,k,l] = 2 cosh(b)^(2 - n/2) sinh(b)^(n/2) for even n = i+j+k+l, else 0
    T = tensors.ising(beta)
    c, s = math.cosh(beta), math.sinh(beta)
    for idx in np.ndindex(2, 2, 2, 2):
        n = sum(idx)
        want = 2 * c ** (2 - n / 2) * s ** (n / 2) if n % 2 == 0 else 0.0
        assert T[idx] == pytest.approx(want, rel=1e-14, abs=1e-15)


@pytest.mark.parametrize("beta", [0.2, 0.5])
def test_ising_one_site_torus(beta):
    # one spin whose two bonds both close on itself: Z = 2 e^(2 beta)
    T = tensors.ising(beta)
    assert np.einsum("ijij->", T) == pytest.approx(2 * math.exp(2 * beta), rel=1e-14)


def test_ising_bond_weight():
    # contracting the shared leg of two neighbours' factors gives e^(beta s s')
    beta = 0.37
    c, s = math.sqrt(math.cosh(beta)), math.sqrt(math.sinh(beta))
    Q = np.array([[c, s], [c, -s]])
    W = Q @ Q.T
    assert W[0, 0] == pytest.approx(math.exp(beta), rel=1e-15)
    assert W[0, 1] == pytest.approx(math.exp(-beta), rel=1e-15)


@pytest.mark.parametrize("beta,n_max", [(0.8, 3), (1.1, 5)])
def test_xy_charge_conservation_and_values(beta, n_max):
    T = tensors.xy(beta, n_max)
    D = 2 * n_max + 1
    n = np.arange(-n_max, n_max + 1)
    for a, b, c, d in np.ndindex(D, D, D, D):
        if n[a] + n[b] != n[c] + n[d]:
            assert T[a, b, c, d] == 0.0
        else:
            want = math.sqrt(iv(n[a], beta) * iv(n[b], beta) * iv(n[c], beta) * iv(n[d], beta))
            assert T[a, b, c, d] == pytest.approx(want, rel=1e-14)


def test_xy_one_site_torus():
    # a site with both bonds closed on itself: Z = e^(2 beta) (cos 0 = 1),
    # reached as n_max grows; the character sum gives (sum_n I_n)^2
    beta = 0.9
    for n_max, tol in [(3, 5e-3), (12, 1e-13)]:
        T = tensors.xy(beta, n_max)
        assert np.einsum("ijij->", T) == pytest.approx(math.exp(2 * beta), rel=tol)


@pytest.mark.parametrize("q", [2, 3, 4])
def test_potts_one_site_torus(q):
    beta = 0.6
    T = tensors.potts(beta, q)
    # sum_sigma W[sigma, sigma]^2 = q e^(2 beta)
    assert np.einsum("ijij->", T) == pytest.approx(q * math.exp(2 * beta), rel=1e-13)


@pytest.mark.parametrize("beta", [0.4, 1.1])
def test_gxy_at_delta_one_is_xy(beta):
    # Delta = 1 removes the nematic term: I_m(0) = delta_{m,0} leaves c_n = I_n
    assert np.array_equal(tensors.gxy(beta, 1.0, 4), tensors.xy(beta, 4))


@pytest.mark.parametrize("beta,delta", [(0.5, 0.2), (0.9, 0.5), (1.3, 0.8), (1.0, 0.0)])
def test_gxy_weights_are_fourier_coefficients(beta, delta):
    # c_n = (1/2pi) int exp(beta delta cos phi + beta (1-delta) cos 2phi) cos(n phi) dphi,
    # by the trapezoid rule on the periodic integrand (exact to rounding at 512 points)
    N = 512
    phi = 2 * np.pi * np.arange(N) / N
    f = np.exp(beta * delta * np.cos(phi) + beta * (1 - delta) * np.cos(2 * phi))
    c = tensors.gxy_weights(beta, delta, 6)
    for n in range(-6, 7):
        want = np.mean(f * np.cos(n * phi))
        assert c[n + 6] == pytest.approx(want, rel=1e-12, abs=1e-14 * c[6])


def test_gxy_at_delta_zero_has_only_even_charges():
    # Delta = 0: c_n = I_{n/2}(beta) for even n, 0 for odd n
    c = tensors.gxy_weights(0.8, 0.0, 6)
    for n in range(-6, 7):
        want = iv(n // 2, 0.8) if n % 2 == 0 else 0.0
        assert c[n + 6] == pytest.approx(want, rel=1e-15, abs=0.0)
