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
