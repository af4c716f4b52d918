"""Initial site tensors of the 2D square-lattice models (oracle, FP64).

Test infrastructure only (see ``oracle/__init__.py``).

Leg order of every rank-4 site tensor is (left, up, right, down), row-major,
left slowest.  Each tensor sits on one lattice site; the bond between two
neighbouring sites is the shared index.

Pins: ``tests/test_oracle_tensors.py`` (closed forms, 1x1 torus traces) and
``tests/test_oracle_exact.py`` (whole-lattice values against brute force).
"""

import numpy as np
from scipy.special import iv


def ising(beta, J=1.0):
    """Ising tensor with bond dimension 2 (Sec. 3.2; the paper uses bond
    dimension 2 for Ising but does not print the tensor).

    The Boltzmann weight of one bond, W[s, s'] = exp(beta*J*s*s') with
    s, s' in {+1, -1}, is split symmetrically as W = Q Q^T with
    Q[s, 0] = sqrt(cosh(beta J)) and Q[s, 1] = s * sqrt(sinh(beta J)).
    Summing the spin of a site gives T[i,j,k,l] = sum_s Q[s,i]Q[s,j]Q[s,k]Q[s,l].
    Valid for beta*J >= 0 (ferromagnet), which covers every workload here.
    """
    bj = beta * J
    if bj < 0:
        raise ValueError("ising tensor needs beta*J >= 0")
    c, s = np.sqrt(np.cosh(bj)), np.sqrt(np.sinh(bj))
    Q = np.array([[c, s], [c, -s]], dtype=np.float64)
    T = np.zeros((2, 2, 2, 2), dtype=np.float64)
    for spin in range(2):
        q = Q[spin]
        T += np.multiply.outer(np.multiply.outer(q, q), np.multiply.outer(q, q))
    return T


def _charge_tensor(w):
    """T[a,b,c,d] = w[a] w[b] w[c] w[d] where the charges obey
    n_a + n_b = n_c + n_d (index = charge + n_max), zero elsewhere."""
    D = len(w)
    T = np.zeros((D, D, D, D), dtype=np.float64)
    for a in range(D):
        for b in range(D):
            for c in range(D):
                d = a + b - c  # n_d = n_a + n_b - n_c, as an index shift
                if 0 <= d < D:
                    T[a, b, c, d] = w[a] * w[b] * w[c] * w[d]
    return T


def xy(beta, n_max):
    """Classical XY tensor from the character expansion (Sec. 3.1 with
    Delta = 1, h = 0; the paper notes its index range is infinite and must be
    truncated from the start).

    exp(beta cos(theta)) = sum_n I_n(beta) exp(i n theta); with the site
    measure d theta / 2pi the angle integral enforces charge conservation
    n_left + n_up = n_right + n_down.  Each bond weight I_n is split as
    sqrt(I_n) onto its two end tensors.  Charges are kept for |n| <= n_max,
    index m = n + n_max, so the bond dimension is 2*n_max + 1.
    """
    if n_max < 0:
        raise ValueError("n_max must be >= 0")
    n = np.arange(-n_max, n_max + 1)
    return _charge_tensor(np.sqrt(iv(n, beta)))


def gxy_weights(beta, delta, n_max):
    """Character coefficients c_n, |n| <= n_max, of the generalized XY bond
    weight exp(beta*delta*cos(phi) + beta*(1-delta)*cos(2 phi)) (Sec. 3.1,
    Eq. (gXY_ham) with h = 0).

    exp(x cos phi) = sum_k I_k(x) e^{i k phi} and
    exp(y cos 2phi) = sum_m I_m(y) e^{2 i m phi}; the coefficient of e^{i n phi}
    in their product is c_n = sum_m I_{n-2m}(x) I_m(y), x = beta*delta,
    y = beta*(1-delta).  The terms fall off like (x/2)^|k| / |k|! times
    (y/2)^|m| / |m|!, so |m| <= n_max + 40 is exact in FP64 for beta of
    order one.
    """
    if n_max < 0:
        raise ValueError("n_max must be >= 0")
    if not 0.0 <= delta <= 1.0 or beta < 0:
        raise ValueError("need 0 <= delta <= 1 and beta >= 0")
    x, y = beta * delta, beta * (1.0 - delta)
    m = np.arange(-(n_max + 40), n_max + 41)
    c = np.array([np.sum(iv(n - 2 * m, x) * iv(m, y)) for n in range(-n_max, n_max + 1)])
    return c


def gxy(beta, delta, n_max):
    """Generalized XY tensor (Sec. 3.1): the XY construction with the bond
    weights I_n(beta) replaced by the coefficients c_n of ``gxy_weights``
    (delta = 1 is the XY model, delta = 0 the pure nematic coupling)."""
    return _charge_tensor(np.sqrt(gxy_weights(beta, delta, n_max)))


def potts(beta, q):
    """q-state Potts tensor (Sec. 3.3).

    W[a, b] = exp(beta) if a == b else 1; W = L L^T by Cholesky; the site
    tensor joins the four bonds of one spin sigma:
    T[i,j,k,l] = sum_sigma L[sigma,i] L[sigma,j] L[sigma,k] L[sigma,l].
    (The printed formula lists the four factors without the spin sum; the
    sum over the site's spin is the reading that makes a network of these
    tensors equal the Potts partition function.)
    """
    if q < 2:
        raise ValueError("q must be >= 2")
    W = np.ones((q, q)) + (np.exp(beta) - 1.0) * np.eye(q)
    L = np.linalg.cholesky(W)
    T = np.einsum("si,sj,sk,sl->ijkl", L, L, L, L)
    return np.ascontiguousarray(T)
