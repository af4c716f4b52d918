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
    D = 2 * n_max + 1
    n = np.arange(-n_max, n_max + 1)
    w = np.sqrt(iv(n, beta))
    T = np.zeros((D, D, D, D), dtype=np.float64)
    for a in range(D):
        for b in range(D):
            for c in range(D):
                d = a + b - c  # n_d = n_a + n_b - n_c, as an index shift
                if 0 <= d < D:
                    T[a, b, c, d] = w[a] * w[b] * w[c] * w[d]
    return T


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
