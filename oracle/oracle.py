"""CPU FP64 oracle for parallel-tempering Monte Carlo of the smoothed-cubic
random-laser model (Benedetti & Leuzzi, arXiv 2511.13508).

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The arithmetic lives
in ``oracle.c`` (plain C, double precision, no code shared with the HIP
library); this module compiles it with gcc and marshals numpy arrays.

Parity status per function (see oracle.c for the passages each follows):
  philox            pinned: numpy.random.Philox (independent implementation)
  frequencies/terms pinned: brute-force enumeration, comb closed forms
  couplings         pinned: moments / normality of the drawn J
  energy            pinned: tensor-contraction brute force, symmetries
  fields            pinned: finite differences of energy, H = -1/2 sum Re(conj a F)
  pair_dE           pinned: brute-force H(a') - H(a)
  init / move       pinned: beta = 0 closed forms of the constrained law
  pt_run            pinned: high-temperature expansion, importance-sampling
                    reference at small N, swap invariants
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OMEGA_RANDOM = 0
OMEGA_COMB = 1
SPLIT_A, SPLIT_B, SPLIT_C = 1, 2, 4
SPLIT_ALL = 7


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11",
               "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class PTParams(C.Structure):
    _fields_ = [
        ("n_modes", C.c_int32), ("rho", C.c_int32), ("n_terms", C.c_int64),
        ("quads", C.c_void_p), ("J", C.c_void_p),
        ("n_temps", C.c_int32), ("n_reps", C.c_int32), ("temps", C.c_void_p),
        ("run_seed", C.c_uint64), ("sample", C.c_int32), ("shared_pairs", C.c_int32),
        ("swap_interval", C.c_int32), ("resync_interval", C.c_int32), ("renorm_tol", C.c_double),
        ("measure_start", C.c_int32), ("measure_interval", C.c_int32), ("n_bins", C.c_int32),
        ("series_len", C.c_int32), ("n_threads", C.c_int32), ("pad1", C.c_int32),
    ]


class PTState(C.Structure):
    _fields_ = [("a", C.c_void_p), ("E", C.c_void_p), ("temp_of", C.c_void_p),
                ("sweeps_done", C.c_int64), ("swaps_done", C.c_int64)]


_ACC_FIELDS = ["e_n", "e_sum", "e_sq", "y2_sum", "y4_sum", "q_n", "q_sum", "q_sq", "q_4", "hist",
               "acc", "tries", "swap_acc", "swap_tries", "series_e", "series_q", "hist_I", "spectrum"]


class PTAccum(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in _ACC_FIELDS] + [("n_meas", C.c_int64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
            P = C.c_void_p
            L.or_philox4x64.argtypes = [P, P, P]
            L.or_frequencies.argtypes = [C.c_int32, C.c_uint64, C.c_int32, P]
            L.or_graph_terms.argtypes = [C.c_int32, P, C.c_double, C.c_int32, P, C.c_int64]
            L.or_graph_terms.restype = C.c_int64
            L.or_graph_terms_sparse.argtypes = [C.c_int32, P, C.c_double, C.c_int32, C.c_int32, C.c_uint64, P]
            L.or_graph_terms_sparse.restype = C.c_int64
            L.or_default_gamma.argtypes = [C.c_int32]
            L.or_default_gamma.restype = C.c_double
            L.or_couplings.argtypes = [C.c_int32, C.c_uint64, C.c_int64, P]
            L.or_energy.argtypes = [C.c_int64, P, P, P]
            L.or_energy.restype = C.c_double
            L.or_fields.argtypes = [C.c_int32, C.c_int64, P, P, P, P]
            L.or_pair_dE.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int32, C.c_int32, P, P]
            L.or_pair_dE.restype = C.c_double
            L.or_init_copy.argtypes = [C.c_int32, C.c_uint64, C.c_int64, P]
            L.or_init_copy_rho.argtypes = [C.c_int32, C.c_uint64, C.c_int64, C.c_int32, P]
            L.or_pt_init.argtypes = [P, P]
            L.or_pt_run.argtypes = [P, P, P, C.c_int64]
            L.or_pt_run.restype = C.c_double
            _lib = L
    return _lib


def _p(x: np.ndarray):
    return x.ctypes.data_as(C.c_void_p)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64(_p(c), _p(k), _p(out))
    return out


def frequencies(N: int, seed: int, omega_kind: int = OMEGA_RANDOM) -> np.ndarray:
    w = np.zeros(N, dtype=np.float64)
    lib().or_frequencies(N, seed, omega_kind, _p(w))
    return w


def default_gamma(N: int) -> float:
    return lib().or_default_gamma(N)


class Graph:
    """One disorder sample: frequencies, kept terms (p, s, m, n) and couplings."""

    def __init__(self, N: int, seed: int, omega_kind: int = OMEGA_RANDOM, split_mask: int = SPLIT_ALL,
                 gamma: float | None = None, mean_degree: int = 0):
        if N < 4:
            raise ValueError("N must be >= 4")
        self.N, self.seed = N, seed
        self.omega = frequencies(N, seed, omega_kind)
        self.gamma = default_gamma(N) if gamma is None or gamma <= 0 else float(gamma)
        L = lib()
        if mean_degree > 0:
            cap = max(mean_degree * N // 4, 1)
            self.quads = np.zeros((cap, 4), dtype=np.int16)
            c = L.or_graph_terms_sparse(N, _p(self.omega), self.gamma, split_mask, mean_degree, seed, _p(self.quads))
            if c < 0:
                raise ValueError("could not draw the sparse graph's terms")
        else:
            c = L.or_graph_terms(N, _p(self.omega), self.gamma, split_mask, None, 0)
            self.quads = np.zeros((max(c, 1), 4), dtype=np.int16)
            c2 = L.or_graph_terms(N, _p(self.omega), self.gamma, split_mask, _p(self.quads), c)
            assert c2 == c
        self.quads = self.quads[:c].copy()
        self.n_terms = int(c)
        self.J = np.zeros(max(c, 1), dtype=np.float64)
        if c > 0:
            L.or_couplings(N, seed, c, _p(self.J))
        self.J = self.J[:c].copy()


def energy(g: Graph, a: np.ndarray) -> float:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return lib().or_energy(g.n_terms, _p(g.quads), _p(g.J), _p(a))


def fields(g: Graph, a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    F = np.zeros(g.N, dtype=np.complex128)
    lib().or_fields(g.N, g.n_terms, _p(g.quads), _p(g.J), _p(a), _p(F))
    return F


def pair_dE(g: Graph, a: np.ndarray, j: int, k: int, aj_new: complex, ak_new: complex) -> float:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    x = np.array([aj_new.real, aj_new.imag])
    y = np.array([ak_new.real, ak_new.imag])
    return lib().or_pair_dE(g.N, g.n_terms, _p(g.quads), _p(g.J), _p(a), j, k, _p(x), _p(y))


def init_copy(N: int, run_seed: int, copy_id: int, rho: int = 4) -> np.ndarray:
    """beta = 0 draw on the constraint surface sum |a|^rho = N (rho = 4 or 2)."""
    a = np.zeros(N, dtype=np.complex128)
    if rho == 4:
        lib().or_init_copy(N, run_seed, copy_id, _p(a))
    else:
        lib().or_init_copy_rho(N, run_seed, copy_id, rho, _p(a))
    return a


class PT:
    """Parallel tempering of one disorder sample (n_temps baths x n_reps replicas)."""

    def __init__(self, g: Graph, temps, n_reps: int = 2, run_seed: int = 1, sample: int = 0,
                 shared_pairs: bool = False, swap_interval: int = 1, resync_interval: int = 100,
                 renorm_tol: float = 1e-6, measure_start: int = 0, measure_interval: int = 1,
                 n_bins: int = 100, series_len: int = 0, n_threads: int = 0, rho: int = 4):
        if rho not in (2, 4):
            raise ValueError("rho must be 4 (smoothed cubic) or 2 (spherical)")
        self.g = g
        self.temps = np.ascontiguousarray(temps, dtype=np.float64)
        if np.any(np.diff(self.temps) <= 0):
            raise ValueError("temperatures must be strictly ascending")
        T = len(self.temps)
        self.T, self.n_reps, self.R = T, n_reps, T * n_reps
        self.rho = rho
        self.P = PTParams(n_modes=g.N, rho=rho, n_terms=g.n_terms, quads=_p(g.quads).value, J=_p(g.J).value,
                          n_temps=T, n_reps=n_reps, temps=_p(self.temps).value, run_seed=run_seed,
                          sample=sample, shared_pairs=int(shared_pairs), swap_interval=swap_interval,
                          resync_interval=resync_interval, renorm_tol=renorm_tol,
                          measure_start=measure_start, measure_interval=measure_interval,
                          n_bins=n_bins, series_len=series_len, n_threads=n_threads)
        self.a = np.zeros((self.R, g.N), dtype=np.complex128)
        self.E = np.zeros(self.R, dtype=np.float64)
        self.temp_of = np.zeros(self.R, dtype=np.int32)
        self.S = PTState(a=_p(self.a).value, E=_p(self.E).value, temp_of=_p(self.temp_of).value)
        self.acc = {}
        shapes = {"hist": (T, n_bins), "hist_I": (T, n_bins), "spectrum": (T, g.N),
                  "swap_acc": (max(T - 1, 1),), "swap_tries": (max(T - 1, 1),),
                  "series_e": (T, max(series_len, 1)), "series_q": (T, max(series_len, 1))}
        for f in _ACC_FIELDS:
            self.acc[f] = np.zeros(shapes.get(f, (T,)), dtype=np.float64)
        self.A = PTAccum(**{f: _p(self.acc[f]).value for f in _ACC_FIELDS})
        lib().or_pt_init(C.byref(self.P), C.byref(self.S))

    @property
    def sweeps_done(self) -> int:
        return self.S.sweeps_done

    @property
    def n_meas(self) -> int:
        return self.A.n_meas

    def run(self, n_sweeps: int) -> float:
        """Advance n_sweeps; returns the worst relative energy drift at recomputations."""
        return lib().or_pt_run(C.byref(self.P), C.byref(self.S), C.byref(self.A), n_sweeps)

    def copy_at(self, r: int, t: int) -> int:
        """Index of the copy of ladder r currently at temperature index t."""
        idx = np.nonzero(self.temp_of[r * self.T:(r + 1) * self.T] == t)[0]
        return r * self.T + int(idx[0])
