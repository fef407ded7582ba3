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


def summarize(acc: dict, N: int, temps) -> dict:
    """Plain per-temperature disorder averages (sec. III.B, sec. IV) from per-sample
    accumulators with a leading sample axis; errors by jackknife over samples.
    Kurtosis (eq. kurt) with the disorder-averaged mean overlap taken as 0."""
    temps = np.asarray(temps, dtype=np.float64)
    en = acc["e_n"]
    E = acc["e_sum"] / en
    per = {"E": E, "cv": (acc["e_sq"] / en - E ** 2) / temps ** 2 / N, "y2": acc["y2_sum"] / en,
           "y4": acc["y4_sum"] / en}
    out = {}
    for k, v in per.items():
        out[k], out[k + "_err"] = jackknife_mean_err(v)
    qn = acc["q_n"]
    q2 = acc["q_sq"] / qn
    out["q2"], out["q2_err"] = jackknife_mean_err(q2)
    num = acc["q_4"] / qn
    den = q2 - (acc["q_sum"] / qn) ** 2
    S = num.shape[0]
    full = num.mean(0) / den.mean(0) ** 2
    loo = np.array([np.delete(num, i, 0).mean(0) / np.delete(den, i, 0).mean(0) ** 2 for i in range(S)])
    out["kurtosis"] = full
    out["kurtosis_err"] = np.sqrt((S - 1) / S * ((loo - loo.mean(0)) ** 2).sum(0))
    return out


def adaptive_ladder(T_grid, C_grid, T_min, T_max, C=0.6):
    """App. A, eq. PT_Ti: T_i = T_{i-1} / (1 - C / sqrt(C_V(T_i))) until T_i >= T_max,
    the implicit equation solved by bisection on the residual (C_V interpolated
    linearly on the grid, constant beyond it)."""
    cv = lambda T: np.interp(T, T_grid, C_grid)  # noqa: E731
    out = [T_min]
    T = T_min
    while True:
        f = lambda x: x * (1.0 - C / np.sqrt(cv(x))) - T  # noqa: E731
        lo, hi = T, T
        while f(hi) < 0:
            hi *= 1.5
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        x = 0.5 * (lo + hi)
        if x >= T_max:
            break
        out.append(x)
        T = x
    return np.array(out)


def window_means(x):
    """Means over [0,1), [1,2), [2,4), ... (sec. III.B doubling windows)."""
    x = np.asarray(x, dtype=np.float64)
    out, b, e = [], 0, 1
    while b < len(x):
        out.append(x[b:min(e, len(x))].mean())
        b, e = e, 2 * e
    return np.array(out)
