"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module only draws random numbers; it holds none of the method's
arithmetic (no energy, no field, no move, no constraint handling).
"""
from __future__ import annotations

import numpy as np


def random_state(N: int, seed: int, n_copies: int | None = None) -> np.ndarray:
    """Complex standard-normal amplitudes, shape (N,) or (n_copies, N), complex128."""
    rng = np.random.default_rng(seed)
    shape = (N,) if n_copies is None else (n_copies, N)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def random_pairs(N: int, seed: int, n: int) -> np.ndarray:
    """n pairs (j, k) of distinct mode indices."""
    rng = np.random.default_rng(seed)
    j = rng.integers(0, N, size=n)
    k = (j + rng.integers(1, N, size=n)) % N
    return np.stack([j, k], axis=1).astype(np.int32)


def random_complex(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0)


def geometric_temps(t_min: float, t_max: float, n: int) -> np.ndarray:
    """n temperatures geometric in [t_min, t_max], ascending."""
    if n == 1:
        return np.array([t_min])
    return t_min * (t_max / t_min) ** (np.arange(n) / (n - 1))
