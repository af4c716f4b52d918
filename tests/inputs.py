"""Seeded synthetic inputs shared by the oracle checks and the GPU tests.

Holds no arithmetic of the method: only random numbers with fixed seeds.
"""

import numpy as np


def random_tensor(dx, dy, seed, positive=False):
    """A rank-4 array of shape (dx, dy, dx, dy): standard normal entries, or
    uniform in [0.1, 1) with ``positive`` (keeps tori traces positive)."""
    rng = np.random.default_rng(seed)
    if positive:
        return rng.uniform(0.1, 1.0, (dx, dy, dx, dy))
    return rng.standard_normal((dx, dy, dx, dy))


def random_projector(dx, dn, seed):
    """An array of shape (dx, dx, dn) with standard normal entries (the
    contractions do not require orthonormal columns)."""
    return np.random.default_rng(seed).standard_normal((dx, dx, dn))


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds) of n requests of a Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def serving_stream(n, seed):
    """A seeded mix of small FP64 requests for the serving parity test:
    tuples (model, beta, n_max, q, d_cut, n_steps).  Ising at T ~ U[1.5, 3.5],
    XY at beta ~ U[0.6, 1.6] with n_max in {2, 3}, 3-state Potts at
    beta ~ U[0.8, 1.2]; D_cut in {8, 12, 16, 24} (at most 16 for XY / Potts);
    10 to 24 directional steps."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        u = rng.random()
        if u < 0.45:
            out.append(("ising", 1.0 / rng.uniform(1.5, 3.5), 0, 2,
                        int(rng.choice([8, 12, 16, 24])), int(rng.integers(10, 25))))
        elif u < 0.85:
            out.append(("xy", rng.uniform(0.6, 1.6), int(rng.integers(2, 4)), 2,
                        int(rng.choice([8, 12, 16])), int(rng.integers(10, 25))))
        else:
            out.append(("potts", rng.uniform(0.8, 1.2), 0, 3,
                        int(rng.choice([8, 12, 16])), int(rng.integers(10, 25))))
    return out


def graded_gram(n, rank, decay, seed):
    """A seeded symmetric positive semidefinite n x n array G diag(w) G^T of
    the given rank: G standard normal (n x rank), w = 10^(-decay i / rank)
    (graded like a coarse-graining environment's spectrum)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, rank))
    w = 10.0 ** (-decay * np.arange(rank) / rank)
    return (G * w) @ G.T


def orthogonal_with_spectrum(values, seed):
    """Q diag(values) Q^T for a seeded orthogonal Q (QR of a standard normal
    square array, signs fixed by R's diagonal)."""
    n = len(values)
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    return (Q * np.asarray(values, dtype=np.float64)) @ Q.T
