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


def random_constrained_state(N: int, seed: int, n_copies: int | None = None) -> np.ndarray:
    """Complex normal amplitudes scaled onto the surface sum |a|^4 = N."""
    a = random_state(N, seed, n_copies)
    s = np.sum(np.abs(a) ** 4, axis=-1, keepdims=True)
    return a * (N / s) ** 0.25


def random_mlp_params(n_in: int, hidden: int, n_out: int, seed: int, out_scale: float = 0.3) -> np.ndarray:
    """A flat parameter vector W1 [n_in, H], b1, W2 [H, H], b2, W3 [H, n_out], b3 (float32)."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(n_in * hidden) / np.sqrt(n_in), 0.1 * rng.standard_normal(hidden),
             rng.standard_normal(hidden * hidden) / np.sqrt(hidden), 0.1 * rng.standard_normal(hidden),
             out_scale * rng.standard_normal(hidden * n_out) / np.sqrt(hidden), 0.1 * rng.standard_normal(n_out)]
    return np.concatenate(parts).astype(np.float32)
