"""Seeded synthetic inputs shared by the oracle side and the HIP side.

Holds none of the method's arithmetic: only random points on the simplex.
"""
import numpy as np


def simplex_points(M, count, seed):
    """Dirichlet(1,...,1) points, shape (count, M)."""
    return np.random.default_rng(seed).dirichlet(np.ones(M), count)


def boundary_points(M, count, seed, lam=1e-6):
    """Points with a random nonempty proper subset of coordinates scaled by
    lam and renormalised (near a sector boundary / singular face)."""
    rng = np.random.default_rng(seed)
    z = rng.dirichlet(np.ones(M), count)
    for i in range(count):
        k = rng.integers(1, M)
        idx = rng.choice(M, size=k, replace=False)
        z[i, idx] *= lam
        z[i] /= z[i].sum()
    return z
