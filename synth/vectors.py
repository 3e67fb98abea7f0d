"""Seeded random input vectors (numpy PCG64), uniform on [-1, 1)."""
import numpy as np


def random_vector(D: int, seed: int, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.random(D) * 2.0 - 1.0).astype(dtype)
