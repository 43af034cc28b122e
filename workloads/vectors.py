"""Seeded random vectors (inputs only)."""
import numpy as np


def gaussian_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """b ~ N(0, 1) drawn in float64 by numpy's default generator, then cast."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def unit_direction(n: int, seed: int) -> np.ndarray:
    """A float64 random direction of unit 2-norm (finite-difference probes)."""
    v = np.random.default_rng(seed).standard_normal(n)
    return v / np.linalg.norm(v)
