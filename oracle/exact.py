"""Exact values used to pin the oracle (closed forms and brute force).

Test infrastructure only (see ``oracle/__init__.py``).

* ``onsager_hyper``    -- the free energy as printed in Sec. 3.2 (generalised
                          hypergeometric 4F3 form), via mpmath.
* ``onsager_integral`` -- Onsager's solution in its one-dimensional integral
                          form (textbook), independent of the 4F3 form.
* ``onsager_tc``       -- the closed value at the critical point,
                          ln(2)/2 + 2G/pi with Catalan's constant G.
* ``onsager_energy``   -- the internal energy per site in closed form
                          (complete elliptic integral of the first kind).
* ``onsager_specific_heat`` -- beta^2 d^2(-beta f)/d beta^2 of the 4F3 form,
                          differentiated by mpmath at 40 digits.
* ``ising_torus``      -- brute-force ln Z / N of the Ising model on an
                          Lx-by-Ly torus by a row transfer matrix.
* ``xy_torus``         -- ln Z / N of the XY model on a tiny torus, the site
                          angles discretised on an M-point uniform grid
                          (exact up to Fourier coefficients of order M).

Temperature convention: k_B = J = 1, beta = 1/T; ln Z / N = -beta f.
"""

import itertools
import math

import numpy as np
from scipy.integrate import quad

TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))


def onsager_hyper(beta, dps=30):
    """-beta f = ln(2 cosh 2beta) - kappa^2 4F3(1,1,3/2,3/2; 2,2,2; 16 kappa^2)
    with kappa = sinh(2beta) / (2 cosh^2(2beta))  (Sec. 3.2, exact free
    energy of the 2D Ising model)."""
    import mpmath as mp

    with mp.workdps(dps):
        b = mp.mpf(beta)
        kap = mp.sinh(2 * b) / (2 * mp.cosh(2 * b) ** 2)
        F = mp.hyper([1, 1, mp.mpf(3) / 2, mp.mpf(3) / 2], [2, 2, 2], 16 * kap**2)
        return float(mp.log(2 * mp.cosh(2 * b)) - kap**2 * F)


def onsager_integral(beta):
    """-beta f = ln(2 cosh 2beta) + (1/2pi) int_0^pi ln[(1 + sqrt(1 - k^2
    sin^2 phi)) / 2] dphi, with k = 2 sinh(2beta) / cosh^2(2beta)
    (Onsager 1944, in the single-integral form of standard texts)."""
    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2

    def f(phi):
        return math.log((1.0 + math.sqrt(max(0.0, 1.0 - (k * math.sin(phi)) ** 2))) / 2.0)

    val, _ = quad(f, 0.0, math.pi, epsabs=1e-15, epsrel=1e-15, limit=400,
                  points=[math.pi / 2])
    return math.log(2.0 * math.cosh(2 * beta)) + val / (2.0 * math.pi)


def onsager_energy(beta):
    """Internal energy per site u = -d(ln Z/N)/d beta of the 2D Ising model:
    u = -coth(2beta) [1 + (2/pi)(2 tanh^2(2beta) - 1) K(k)],
    k = 2 sinh(2beta) / cosh^2(2beta), K the complete elliptic integral of
    the first kind of modulus k (Onsager 1944, as in standard texts).
    u -> 0 as beta -> 0 and u -> -2 as beta -> infinity."""
    from scipy.special import ellipk

    t = math.tanh(2 * beta)
    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    return -(1.0 / t) * (1.0 + (2.0 / math.pi) * (2.0 * t * t - 1.0) * float(ellipk(k * k)))


def onsager_specific_heat(beta, dps=40):
    """Specific heat per site c = beta^2 d^2(ln Z/N)/d beta^2 from the 4F3
    form of ``onsager_hyper``, differentiated by mpmath at ``dps`` digits
    (away from T_c, where c diverges logarithmically)."""
    import mpmath as mp

    with mp.workdps(dps):
        def f(b):
            kap = mp.sinh(2 * b) / (2 * mp.cosh(2 * b) ** 2)
            F = mp.hyper([1, 1, mp.mpf(3) / 2, mp.mpf(3) / 2], [2, 2, 2], 16 * kap**2)
            return mp.log(2 * mp.cosh(2 * b)) - kap**2 * F

        b = mp.mpf(beta)
        return float(b * b * mp.diff(f, b, 2))


def onsager_tc():
    """-beta_c f at T_c = 2 / ln(1 + sqrt 2): ln(2)/2 + 2G/pi."""
    G = 0.915965594177219015054603514932384110774  # Catalan's constant
    return math.log(2.0) / 2.0 + 2.0 * G / math.pi


def ising_torus(beta, Lx, Ly):
    """Brute-force ln Z / N of the Ising model (J = 1, h = 0) on an Lx-by-Ly
    torus.  Bonds: each site to its right neighbour (x+1 mod Lx) and to its
    lower neighbour (y+1 mod Ly), so a length-1 direction gives a self bond
    (weight e^beta) and a length-2 direction gives two distinct bonds.
    Z = Tr(A^Ly) with the row-to-row transfer matrix A."""
    rows = np.array(list(itertools.product([1, -1], repeat=Lx)), dtype=np.float64)
    # energy inside a row, with periodic wrap
    e_in = np.array([sum(r[x] * r[(x + 1) % Lx] for x in range(Lx)) for r in rows])
    # energy between consecutive rows r -> r'
    e_between = rows @ rows.T
    A = np.exp(beta * (e_in[:, None] + e_between))
    # ln Tr(A^Ly) by scaled powers
    P = np.eye(A.shape[0])
    logscale = 0.0
    for _ in range(Ly):
        P = P @ A
        m = np.abs(P).max()
        P /= m
        logscale += math.log(m)
    return (logscale + math.log(np.trace(P))) / (Lx * Ly)


def xy_torus(beta, Lx, Ly, M=48):
    """ln Z / N of the classical XY model, H = -sum cos(theta_i - theta_j),
    on an Lx-by-Ly torus with site measure d theta / 2pi.  Bonds as in
    ``ising_torus``.  The angles take the M values 2 pi m / M; the grid sum
    equals the integral up to Fourier modes of order M of the integrand,
    whose size is about I_M(Lx*Ly*4*beta) / I_0 -- negligible for M = 48
    and the small beta used here.  Z = Tr(A^Ly) with the row transfer
    matrix A over M**Lx row states."""
    th = 2.0 * math.pi * np.arange(M) / M
    rows = np.array(list(itertools.product(range(M), repeat=Lx)))
    ang = th[rows]                                         # (M^Lx, Lx)
    e_in = np.cos(ang - np.roll(ang, -1, axis=1)).sum(axis=1)
    e_between = np.cos(ang[:, None, :] - ang[None, :, :]).sum(axis=2)
    A = np.exp(beta * (e_in[:, None] + e_between)) / (M ** Lx)
    P = np.eye(A.shape[0])
    logscale = 0.0
    for _ in range(Ly):
        P = P @ A
        m = np.abs(P).max()
        P /= m
        logscale += math.log(m)
    return (logscale + math.log(np.trace(P))) / (Lx * Ly)


def xy_high_temperature(beta):
    """Leading terms of the high-temperature (small beta) expansion of the
    XY free energy per site on the infinite square lattice:
    -beta f = 2 ln I0(beta) + 2 t^4 + O(t^6), t = I1(beta)/I0(beta)
    (character expansion: the smallest closed charge loop is an elementary
    plaquette, weight t^4, in both orientations)."""
    from scipy.special import iv

    t = iv(1, beta) / iv(0, beta)
    return 2.0 * math.log(iv(0, beta)) + 2.0 * t**4, t
