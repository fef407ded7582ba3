"""Plain reference estimators for the analysis step (test infrastructure only).

tau_int: integrated autocorrelation time with Sokal's automatic windowing
(A. D. Sokal, "Monte Carlo methods in statistical mechanics: foundations and
new algorithms", 1996): tau(W) = 1/2 + sum_{t=1..W} rho(t), with the smallest
W such that W >= c * tau(W).  Pinned against the AR(1) closed form
tau = (1 + phi) / (2 (1 - phi)) and tau = 1/2 for i.i.d. data.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(x: np.ndarray) -> np.ndarray:
    """rho(t) = C(t)/C(0), C(t) = (1/n) sum_i (x_i - m)(x_{i+t} - m), by direct sums."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    d = x - x.mean()
    c = np.array([np.dot(d[: n - t], d[t:]) / n for t in range(n)])
    return c / c[0] if c[0] > 0 else np.zeros(n)


def tau_int(x, c_window: float = 6.0):
    rho = autocorrelation(x)
    tau = 0.5
    W = 0
    for t in range(1, len(rho)):
        tau += rho[t]
        W = t
        if t >= c_window * tau:
            break
    return tau, W


def jackknife_mean_err(values: np.ndarray):
    """Mean and jackknife error over the first axis (one value per disorder sample)."""
    v = np.asarray(values, dtype=np.float64)
    n = v.shape[0]
    loo = (v.sum(axis=0) - v) / (n - 1)
    m = loo.mean(axis=0)
    return v.mean(axis=0), np.sqrt((n - 1) / n * ((loo - m) ** 2).sum(axis=0))
