"""Independent references that pin the oracle (test code only).

Each helper reaches a quantity of the method by a route different from the
oracle's: enumeration with itertools, contraction of a dense coupling tensor,
i.i.d. sampling of the infinite-temperature law, closed forms.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def numpy_philox_block(ctr, key) -> np.ndarray:
    """Philox4x64-10 block at counter ``ctr`` via numpy's own implementation.

    numpy advances its 256-bit counter by one before producing a block, so it is
    started at ctr - 1 (mod 2^256)."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    start = np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    return bg.random_raw(4)


def enumerate_terms(omega: np.ndarray, gamma: float, split_mask: int = 7):
    """All kept (p, s, m, n) terms: every 4-subset, every split into a
    conjugated pair and a plain pair whose frequency sums differ by < gamma.
    Order: subsets lexicographic, then splits (i,l|j,k), (i,k|j,l), (i,j|k,l)."""
    out = []
    for i, j, k, l in itertools.combinations(range(len(omega)), 4):
        for bit, (p, s, m, n) in zip((1, 2, 4), ((i, l, j, k), (i, k, j, l), (i, j, k, l))):
            if split_mask & bit and abs((omega[p] + omega[s]) - (omega[m] + omega[n])) < gamma:
                out.append((p, s, m, n))
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def coupling_tensor(N: int, quads: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Dense T[k1,k2,k3,k4] with H = -sum T conj(a_k1) a_k2 conj(a_k3) a_k4 + c.c.
    (the index form of the 4-body Hamiltonian in the paper): each kept monomial
    conj(a_p) conj(a_s) a_m a_n appears at the four placements of {p,s} on the
    conjugated slots and {m,n} on the plain slots, each with weight J/4."""
    T = np.zeros((N, N, N, N))
    for (p, s, m, n), j in zip(quads, J):
        for k1, k3 in ((p, s), (s, p)):
            for k2, k4 in ((m, n), (n, m)):
                T[k1, k2, k3, k4] += j / 4.0
    return T


def energy_tensor(T: np.ndarray, a: np.ndarray) -> float:
    ac = np.conj(a)
    x = np.einsum("abcd,a,b,c,d->", T, ac, a, ac, a)
    return float(-(x + np.conj(x)).real)


def energy_batch(quads: np.ndarray, J: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Energies of a batch a[M, N] (used as a tool by the sampling references)."""
    p, s, m, n = (quads[:, i] for i in range(4))
    X = np.conj(a[:, p]) * np.conj(a[:, s]) * a[:, m] * a[:, n]
    return -2.0 * (X.real @ J)


def beta0_draw(N: int, M: int, rng: np.random.Generator) -> np.ndarray:
    """M i.i.d. configurations of the infinite-temperature law on sum |a|^4 = N:
    intensities uniform on the positive part of the sphere sum u^2 = N
    (u = sqrt(N) |g| / ||g||), phases uniform."""
    g = rng.standard_normal((M, N))
    u = math.sqrt(N) * np.abs(g) / np.linalg.norm(g, axis=1, keepdims=True)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(M, N))
    return np.sqrt(u) * np.exp(1j * ph)


def beta0_draw_sphere(N: int, M: int, rng: np.random.Generator) -> np.ndarray:
    """M i.i.d. configurations of the infinite-temperature law on the complex
    sphere sum |a|^2 = N: a = sqrt(N) z / ||z|| with z complex standard normal."""
    z = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    return math.sqrt(N) * z / np.linalg.norm(z, axis=1, keepdims=True)


def beta0_moments_sphere(N: int) -> dict:
    """Closed forms on the complex sphere: the intensities are N times a flat
    Dirichlet vector, so |a|^2 / N ~ Beta(1, N - 1) with E x^m = m! (N-1)! / (N+m-1)!;
    q = Re <a, b> / N is the cosine of two independent uniform directions of
    R^(2N), variance 1 / (2N)."""
    return {
        "E|a|^2": 1.0,
        "E|a|^4": 2.0 * N / (N + 1.0),
        "E|a|^8": 24.0 * N ** 3 / ((N + 1.0) * (N + 2.0) * (N + 3.0)),
        "Var q": 1.0 / (2.0 * N),
    }


def var0_energy_sphere(N: int, J: np.ndarray) -> float:
    """Var of H at infinite temperature on the sphere: 2 sum J^2 E[I_p I_s I_m I_n]
    with E[I_p I_s I_m I_n] = N^4 (N-1)! / (N+3)!."""
    return 2.0 * N ** 3 / ((N + 1.0) * (N + 2.0) * (N + 3.0)) * float(np.sum(J ** 2))


def beta0_moments(N: int) -> dict:
    """Closed forms at infinite temperature.  The intensities are
    u_k = |a_k|^2 = sqrt(N) |g_k| / ||g|| for a standard normal g in R^N, so with
    ||g|| independent of the direction g / ||g||: E u_k = sqrt(N) E|g_k| / E||g||,
    E u_k^2 = 1 and, for k != l, E u_k u_l = N E|g_k| E|g_l| / E||g||^2 = 2 / pi.
    The total intensity per mode x = I / N = (1/N) sum_k u_k then has
    E x = E u_k and E x^2 = (N E u^2 + N (N - 1) (2 / pi)) / N^2."""
    ex1 = math.exp(math.lgamma(N / 2) - math.lgamma((N + 1) / 2)) / math.sqrt(math.pi)
    return {
        "E|a|^2": math.sqrt(N) * ex1,
        "E|a|^4": 1.0,
        "E|a|^8": 3.0 * N / (N + 2.0),
        "Var q": ex1 * ex1 / 2.0,
        "E I/N": math.sqrt(N) * ex1,
        "E (I/N)^2": (N + N * (N - 1) * 2.0 / math.pi) / N ** 2,
    }


def var0_energy(N: int, J: np.ndarray) -> float:
    """Var of H at infinite temperature: 8N / (pi^2 (N+2)) * sum J^2."""
    return 8.0 * N / (math.pi ** 2 * (N + 2.0)) * float(np.sum(J ** 2))


def comb_count(N: int) -> int:
    """Number of i<j<k<l with i+l = j+k (the comb's kept terms)."""
    if N % 2 == 0:
        return N * (N - 2) * (2 * N - 5) // 24
    return (N - 1) * (N - 3) * (2 * N - 1) // 24


def importance_reference(quads, J, N, temps, M, seed, chunk=200000, draw=None, i_bins=0):
    """Thermal averages at each temperature by reweighting i.i.d. infinite-
    temperature draws: <O>_beta = E0[O w] / E0[w], w = exp(-beta H).  Two
    independent draws give the overlap.  Returns (mean, stderr) dicts of
    arrays over temps; the error is the delta-method error of a ratio
    estimator, sqrt(sum w^2 (O - mean)^2) / sum w.  i_bins > 0 adds "pI":
    the probability of each of i_bins equal bins of I / N on [0, 1] (shape
    [temps][i_bins])."""
    rng = np.random.default_rng(seed)
    draw = draw or beta0_draw
    cols = {k: [] for k in ("Ha", "Hb", "y2", "y4", "q", "x")}
    for start in range(0, M, chunk):
        m = min(chunk, M - start)
        a = draw(N, m, rng)
        b = draw(N, m, rng)
        cols["Ha"].append(energy_batch(quads, J, a))
        cols["Hb"].append(energy_batch(quads, J, b))
        I = np.sum(np.abs(a) ** 2, axis=1)
        S2 = np.sum(np.abs(a) ** 4, axis=1)
        S4 = np.sum(np.abs(a) ** 8, axis=1)
        cols["y2"].append(S2 / I ** 2)
        cols["y4"].append(S4 / S2 ** 2)
        cols["q"].append(np.sum(np.conj(a) * b, axis=1).real / N)
        cols["x"].append(I / N)
    Ha, Hb, y2, y4, q, x = (np.concatenate(cols[k]) for k in ("Ha", "Hb", "y2", "y4", "q", "x"))

    def ratio(w, O):
        r = np.sum(w * O) / np.sum(w)
        return r, math.sqrt(np.sum(w ** 2 * (O - r) ** 2)) / np.sum(w)

    mean = {k: [] for k in ("E", "E2", "y2", "y4", "q2", "q4", "x")}
    err = {k: [] for k in mean}
    if i_bins:
        xb = np.clip(np.floor(x * i_bins).astype(np.int64), 0, i_bins - 1)
        mean["pI"], err["pI"] = [], []
    for T in temps:
        beta = 1.0 / T
        la, lb = -beta * Ha, -beta * Hb
        wa = np.exp(la - la.max())
        wb = np.exp(lb - lb.max())
        for k, w, O in (("E", wa, Ha), ("E2", wa, Ha ** 2), ("y2", wa, y2), ("y4", wa, y4),
                        ("q2", wa * wb, q ** 2), ("q4", wa * wb, q ** 4), ("x", wa, x)):
            r, e = ratio(w, O)
            mean[k].append(r)
            err[k].append(e)
        if i_bins:
            pr = [ratio(wa, (xb == b).astype(np.float64)) for b in range(i_bins)]
            mean["pI"].append([v[0] for v in pr])
            err["pI"].append([v[1] for v in pr])
    return ({k: np.array(v) for k, v in mean.items()}, {k: np.array(v) for k, v in err.items()})
