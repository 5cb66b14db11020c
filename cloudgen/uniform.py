"""Uniform random points in a cube: the synthetic cloud of 1 M random points
on which Section 3.5 compares density growth with monotonic growth of the
k-NN search radius (its side is not stated; 100 m gives one point per cubic
metre)."""
import numpy as np


def uniform_cube(seed=7, n=1_000_000, side=100.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, side, (n, 3))
