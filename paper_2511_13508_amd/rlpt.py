"""Python binding of librlpt (argument marshalling only).

Every computation runs in librlpt.so: the host graph builder in C++ and the
Monte Carlo path in HIP kernels for gfx950.  PyTorch provides the device
workspace and the stream.  Names follow the C ABI in include/rlpt.h.
Importing this module does not need a GPU; creating a context does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlpt.so")

RLPT_OK, RLPT_E_ARG, RLPT_E_NOMEM, RLPT_E_HIP, RLPT_E_STATE, RLPT_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
OMEGA_RANDOM, OMEGA_COMB = 0, 1
SPLIT_A, SPLIT_B, SPLIT_C, SPLIT_ALL = 1, 2, 4, 7
FP32, FP64 = 0, 1
LAYOUT_AUTO, LAYOUT_PACKED, LAYOUT_CHUNKED = 0, 1, 2
FIELDS_STREAM, FIELDS_CACHED = 0, 1
ABI_VERSION = 4

# every symbol declared in include/rlpt.h
EXPORTS = [
    "rlpt_abi_version", "rlpt_last_error", "rlpt_graph_build", "rlpt_graph_free", "rlpt_graph_info_get",
    "rlpt_graph_export", "rlpt_config_default", "rlpt_workspace_size", "rlpt_create", "rlpt_destroy",
    "rlpt_init", "rlpt_sweep", "rlpt_swap", "rlpt_resync", "rlpt_check", "rlpt_run_graph", "rlpt_sweep_timing",
    "rlpt_sweep_time_get", "rlpt_counters", "rlpt_stream_lists",
    "rlpt_get_state", "rlpt_set_state", "rlpt_get_energies", "rlpt_energy_fp64", "rlpt_energy_fp64_noalloc",
    "rlpt_local_fields",
    "rlpt_pair_dE", "rlpt_observables", "rlpt_tau_int", "rlpt_tune_clear", "rlpt_tune_set", "rlpt_tune_get",
    "rlpt_tune_save", "rlpt_tune_load", "rlpt_autotune", "rlpt_tile_of", "rlpt_mlp_setup", "rlpt_mlp_n_params",
    "rlpt_mlp_set_params", "rlpt_mlp_get_params", "rlpt_mlp_set_pairs", "rlpt_mlp_harvest", "rlpt_mlp_train",
    "rlpt_mlp_forward", "rlpt_mlp_loss_grad", "rlpt_mlp_infer", "rlpt_mlp_enable", "rlpt_mlp_move", "rlpt_mlp_stats",
    "rlpt_mlp_last_move", "rlpt_summarize", "rlpt_adaptive_ladder", "rlpt_window_means",
    "rlpt_checkpoint_save", "rlpt_checkpoint_load"]


class RlptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librlpt error {code}: {msg}")
        self.code = code


class Tile(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("precision", C.c_int32), ("shared_pairs", C.c_int32),
                ("block_threads", C.c_int32), ("copies_per_block", C.c_int32), ("pad", C.c_int32),
                ("ms_per_sweep", C.c_double)]


class GraphDesc(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("omega_kind", C.c_int32), ("seed", C.c_uint64),
                ("split_mask", C.c_int32), ("mean_degree", C.c_int32), ("gamma", C.c_double)]


class GraphInfo(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("pad", C.c_int32), ("n_terms", C.c_int64), ("deg_min", C.c_int64),
                ("deg_max", C.c_int64), ("deg_sum", C.c_int64), ("gamma", C.c_double), ("sigma2", C.c_double),
                ("list_entries", C.c_int64), ("list_bytes", C.c_int64), ("chunk_entries", C.c_int64),
                ("chunk_bytes", C.c_int64), ("pair_entries", C.c_int64), ("gather_entries", C.c_int64)]


class Config(C.Structure):
    _fields_ = [("n_temps", C.c_int32), ("n_reps", C.c_int32), ("precision", C.c_int32),
                ("shared_pairs", C.c_int32), ("swap_interval", C.c_int32), ("resync_interval", C.c_int32),
                ("renorm_tol", C.c_double), ("drift_tol", C.c_double), ("measure_start", C.c_int32),
                ("measure_interval", C.c_int32), ("n_bins", C.c_int32), ("series_len", C.c_int32),
                ("block_threads", C.c_int32), ("copies_per_block", C.c_int32), ("list_layout", C.c_int32),
                ("mlp_nets", C.c_int32), ("mlp_hidden", C.c_int32), ("mlp_components", C.c_int32),
                ("mlp_capacity", C.c_int32), ("mlp_batch", C.c_int32), ("field_mode", C.c_int32),
                ("rho", C.c_int32), ("mlp_subset", C.c_int32)]


OBS_FIELDS = ["e_n", "e_sum", "e_sq", "y2_sum", "y4_sum", "q_n", "q_sum", "q_sq", "q_4", "hist", "acc", "tries",
              "swap_acc", "swap_tries", "series_e", "series_q", "hist_I", "spectrum"]


class Obs(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in OBS_FIELDS]


_lib = None


def lib() -> C.CDLL:
    """Load librlpt.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"librlpt.so not built at {LIB_PATH}; run `python -m paper_2511_13508_amd.build`")
    # torch bundles its own HIP runtime with the same soname; load it first so
    # that librlpt binds to that one runtime instead of pulling in a second
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "rlpt_abi_version": ([], C.c_int),
        "rlpt_checkpoint_save": ([P, C.c_char_p], C.c_int),
        "rlpt_checkpoint_load": ([P, C.c_char_p], C.c_int),
        "rlpt_last_error": ([], C.c_char_p),
        "rlpt_graph_build": ([P, P], C.c_int),
        "rlpt_graph_free": ([P], None),
        "rlpt_graph_info_get": ([P, P], C.c_int),
        "rlpt_graph_export": ([P, P, P, P], C.c_int),
        "rlpt_config_default": ([P], C.c_int),
        "rlpt_workspace_size": ([P, P, i32, P], C.c_int),
        "rlpt_create": ([P, P, i32, P, P, C.c_size_t, P, P], C.c_int),
        "rlpt_destroy": ([P], C.c_int),
        "rlpt_init": ([P, u64], C.c_int),
        "rlpt_sweep": ([P, i32], C.c_int),
        "rlpt_swap": ([P], C.c_int),
        "rlpt_resync": ([P, P], C.c_int),
        "rlpt_check": ([P], C.c_int),
        "rlpt_run_graph": ([P, i32, i32], C.c_int),
        "rlpt_sweep_timing": ([P, i32], C.c_int),
        "rlpt_sweep_time_get": ([P, P, P], C.c_int),
        "rlpt_counters": ([P, P, P, P], C.c_int),
        "rlpt_stream_lists": ([P, i32, P], C.c_int),
        "rlpt_get_state": ([P, i32, i32, P], C.c_int),
        "rlpt_set_state": ([P, i32, i32, P], C.c_int),
        "rlpt_get_energies": ([P, P, P], C.c_int),
        "rlpt_energy_fp64": ([P, P], C.c_int),
        "rlpt_energy_fp64_noalloc": ([P, P], C.c_int),
        "rlpt_local_fields": ([P, i32, P], C.c_int),
        "rlpt_pair_dE": ([P, i32, i32, P, P, P, P, P], C.c_int),
        "rlpt_observables": ([P, P], C.c_int),
        "rlpt_tau_int": ([P, i64, d, P, P], C.c_int),
        "rlpt_tune_clear": ([], C.c_int),
        "rlpt_tune_set": ([P], C.c_int),
        "rlpt_tune_get": ([P, i32, P], C.c_int),
        "rlpt_tune_save": ([C.c_char_p], C.c_int),
        "rlpt_tune_load": ([C.c_char_p], C.c_int),
        "rlpt_autotune": ([P, P, i32, P, P, C.c_size_t, P, i32, P], C.c_int),
        "rlpt_tile_of": ([P, P, P], C.c_int),
        "rlpt_mlp_setup": ([P, P, u64], C.c_int),
        "rlpt_mlp_n_params": ([P, P, P], C.c_int),
        "rlpt_mlp_set_params": ([P, i32, P], C.c_int),
        "rlpt_mlp_get_params": ([P, i32, P], C.c_int),
        "rlpt_mlp_set_pairs": ([P, i32, i32, P, P], C.c_int),
        "rlpt_mlp_harvest": ([P, i32, i32], C.c_int),
        "rlpt_mlp_train": ([P, i32, d, P], C.c_int),
        "rlpt_mlp_forward": ([P, i32, i32, P], C.c_int),
        "rlpt_mlp_loss_grad": ([P, i32, P, P], C.c_int),
        "rlpt_mlp_infer": ([P, i32, i32, P, P], C.c_int),
        "rlpt_mlp_enable": ([P, i32, d], C.c_int),
        "rlpt_mlp_move": ([P, d], C.c_int),
        "rlpt_mlp_stats": ([P, P, P], C.c_int),
        "rlpt_mlp_last_move": ([P, i32, P, P, P], C.c_int),
        "rlpt_summarize": ([P, i32, i32, i32, P, P], C.c_int),
        "rlpt_adaptive_ladder": ([P, P, i32, d, d, d, P, i32, P], C.c_int),
        "rlpt_window_means": ([P, i64, P, P, i32, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != RLPT_OK:
        raise RlptError(rc, lib().rlpt_last_error().decode())


def _ptr(x: np.ndarray):
    return x.ctypes.data_as(C.c_void_p)


def abi_version() -> int:
    return lib().rlpt_abi_version()


class Graph:
    """A disorder sample built by rlpt_graph_build (host memory)."""

    def __init__(self, n_modes: int, seed: int, omega_kind: int = OMEGA_RANDOM, split_mask: int = SPLIT_ALL,
                 gamma: float = 0.0, mean_degree: int = 0):
        self._h = C.c_void_p()
        desc = GraphDesc(n_modes=n_modes, omega_kind=omega_kind, seed=seed, split_mask=split_mask, gamma=gamma,
                         mean_degree=mean_degree)
        _check(lib().rlpt_graph_build(C.byref(desc), C.byref(self._h)))
        self.N = n_modes
        self.seed = seed

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.rlpt_graph_free(self._h)
            self._h = None

    def info(self) -> dict:
        inf = GraphInfo()
        _check(lib().rlpt_graph_info_get(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in GraphInfo._fields_ if f != "pad"}

    def export(self):
        inf = self.info()
        c = inf["n_terms"]
        omega = np.zeros(self.N)
        quads = np.zeros((c, 4), dtype=np.int16)
        J = np.zeros(c)
        _check(lib().rlpt_graph_export(self._h, _ptr(omega), _ptr(quads), _ptr(J)))
        return omega, quads, J


def default_config(**kw) -> Config:
    cfg = Config()
    _check(lib().rlpt_config_default(C.byref(cfg)))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


class Context:
    """A parallel-tempering context over a torch-owned device workspace."""

    def __init__(self, graphs, temps, config: Config | None = None, device: str = "cuda:0", stream=None, **kw):
        import torch

        self.graphs = list(graphs)
        self.cfg = config if config is not None else default_config(**kw)
        if config is not None and kw:
            for k, v in kw.items():
                setattr(self.cfg, k, v)
        self.temps = np.ascontiguousarray(temps, dtype=np.float64)
        if len(self.temps) != self.cfg.n_temps:
            raise ValueError("len(temps) must equal config n_temps")
        arr = (C.c_void_p * len(self.graphs))(*[g._h.value for g in self.graphs])
        self._garr = arr
        nbytes = C.c_size_t()
        _check(lib().rlpt_workspace_size(C.byref(self.cfg), arr, len(self.graphs), C.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): HIP graphs cannot capture the null stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._h = C.c_void_p()
        _check(lib().rlpt_create(C.byref(self.cfg), arr, len(self.graphs), _ptr(self.temps),
                                 C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(self._h)))
        self.S = len(self.graphs)
        self.T = self.cfg.n_temps
        self.reps = self.cfg.n_reps
        self.R = self.T * self.reps
        self.n_copies = self.R * self.S
        self.Ns = [g.N for g in self.graphs]

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().rlpt_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def init(self, run_seed: int):
        _check(lib().rlpt_init(self._h, run_seed))

    def sweep(self, n: int):
        _check(lib().rlpt_sweep(self._h, n))

    def swap(self):
        _check(lib().rlpt_swap(self._h))

    def resync(self) -> float:
        d = C.c_double()
        _check(lib().rlpt_resync(self._h, C.byref(d)))
        return d.value

    def check(self):
        _check(lib().rlpt_check(self._h))

    def run_graph(self, n_sweeps: int, n_segments: int):
        _check(lib().rlpt_run_graph(self._h, n_sweeps, n_segments))

    def sweep_timing(self, enable: bool = True):
        _check(lib().rlpt_sweep_timing(self._h, int(enable)))

    def sweep_time(self):
        """(summed sweep-kernel ms, timed launches) since the last call."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().rlpt_sweep_time_get(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def stream_lists(self, n_launches: int = 5) -> float:
        """mean ms per launch of the list-stream ceiling kernel (see the header)"""
        ms = C.c_double()
        _check(lib().rlpt_stream_lists(self._h, n_launches, C.byref(ms)))
        return ms.value

    def tile(self):
        """(threads per workgroup, copies per workgroup of each sample) of the sweep launch."""
        b = C.c_int32()
        cp = np.zeros(self.S, dtype=np.int32)
        _check(lib().rlpt_tile_of(self._h, C.byref(b), _ptr(cp)))
        return b.value, cp

    # ---------------------------------------------------------- learned proposal
    def mlp_setup(self, temp_index, seed: int = 1):
        t = np.ascontiguousarray(temp_index, dtype=np.int32)
        _check(lib().rlpt_mlp_setup(self._h, _ptr(t), seed))

    def mlp_sizes(self):
        n, o = C.c_int64(), C.c_int32()
        _check(lib().rlpt_mlp_n_params(self._h, C.byref(n), C.byref(o)))
        return n.value, o.value

    def mlp_set_params(self, net: int, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().rlpt_mlp_set_params(self._h, net, _ptr(p)))

    def mlp_get_params(self, net: int) -> np.ndarray:
        p = np.zeros(self.mlp_sizes()[0], dtype=np.float32)
        _check(lib().rlpt_mlp_get_params(self._h, net, _ptr(p)))
        return p

    def mlp_set_pairs(self, net: int, before, after):
        b = np.ascontiguousarray(before, dtype=np.complex128)
        a = np.ascontiguousarray(after, dtype=np.complex128)
        _check(lib().rlpt_mlp_set_pairs(self._h, net, b.shape[0], _ptr(b), _ptr(a)))

    def mlp_harvest(self, rounds: int, lag: int = 1):
        _check(lib().rlpt_mlp_harvest(self._h, rounds, lag))

    def mlp_train(self, steps: int, lr: float = 1e-3) -> np.ndarray:
        L = np.zeros(self.cfg.mlp_nets)
        _check(lib().rlpt_mlp_train(self._h, steps, lr, _ptr(L)))
        return L

    def mlp_forward(self, net: int, n: int) -> np.ndarray:
        out = np.zeros((n, self.mlp_sizes()[1]))
        _check(lib().rlpt_mlp_forward(self._h, net, n, _ptr(out)))
        return out

    def mlp_loss_grad(self, net: int):
        L = C.c_double()
        g = np.zeros(self.mlp_sizes()[0], dtype=np.float32)
        _check(lib().rlpt_mlp_loss_grad(self._h, net, C.byref(L), _ptr(g)))
        return L.value, g

    def mlp_infer(self, net: int, states) -> np.ndarray:
        a = np.ascontiguousarray(states, dtype=np.complex128)
        out = np.zeros((a.shape[0], self.mlp_sizes()[1]))
        _check(lib().rlpt_mlp_infer(self._h, net, a.shape[0], _ptr(a), _ptr(out)))
        return out

    def mlp_enable(self, moves_per_sweep: int, step_scale: float = 1.0):
        _check(lib().rlpt_mlp_enable(self._h, moves_per_sweep, step_scale))

    def mlp_move(self, step_scale: float = 1.0):
        _check(lib().rlpt_mlp_move(self._h, step_scale))

    def mlp_stats(self):
        a = np.zeros(self.cfg.mlp_nets)
        t = np.zeros(self.cfg.mlp_nets)
        _check(lib().rlpt_mlp_stats(self._h, _ptr(a), _ptr(t)))
        return a, t

    def mlp_last_move(self, net: int):
        B = self.S * self.reps
        la = np.zeros(B)
        cp = np.zeros(B, dtype=np.int32)
        prop = np.zeros((B, self.Ns[0]), dtype=np.complex128)
        _check(lib().rlpt_mlp_last_move(self._h, net, _ptr(la), _ptr(cp), _ptr(prop)))
        return la, cp, prop

    def counters(self):
        a, b, m = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().rlpt_counters(self._h, C.byref(a), C.byref(b), C.byref(m)))
        return a.value, b.value, m.value

    def _n_complex(self, first, n):
        return sum(self.Ns[c // self.R] for c in range(first, first + n))

    def get_state(self, first: int = 0, n: int | None = None) -> np.ndarray:
        n = self.n_copies - first if n is None else n
        buf = np.zeros(self._n_complex(first, n), dtype=np.complex128)
        _check(lib().rlpt_get_state(self._h, first, n, _ptr(buf)))
        return buf

    def set_state(self, a: np.ndarray, first: int = 0, n: int | None = None):
        a = np.ascontiguousarray(a, dtype=np.complex128).ravel()
        n = self.n_copies - first if n is None else n
        if a.size != self._n_complex(first, n):
            raise ValueError("state size does not match the copy range")
        _check(lib().rlpt_set_state(self._h, first, n, _ptr(a)))

    def energies(self):
        E = np.zeros(self.n_copies)
        t = np.zeros(self.n_copies, dtype=np.int32)
        _check(lib().rlpt_get_energies(self._h, _ptr(E), _ptr(t)))
        return E, t

    def energy_fp64(self) -> np.ndarray:
        E = np.zeros(self.n_copies)
        _check(lib().rlpt_energy_fp64(self._h, _ptr(E)))
        return E

    def energy_fp64_noalloc(self, out) -> None:
        """FP64 energies into a caller-owned float64 device tensor `out` of
        n_copies elements, asynchronously on the context's stream (the library
        allocates nothing; see the header)."""
        import torch
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous() and out.numel() >= self.n_copies
        _check(lib().rlpt_energy_fp64_noalloc(self._h, C.c_void_p(out.data_ptr())))

    def checkpoint_save(self, path: str):
        _check(lib().rlpt_checkpoint_save(self._h, str(path).encode()))

    def checkpoint_load(self, path: str):
        _check(lib().rlpt_checkpoint_load(self._h, str(path).encode()))

    def local_fields(self, copy: int) -> np.ndarray:
        F = np.zeros(self.Ns[copy // self.R], dtype=np.complex128)
        _check(lib().rlpt_local_fields(self._h, copy, _ptr(F)))
        return F

    def pair_dE(self, copy: int, j, k, aj_new, ak_new) -> np.ndarray:
        j = np.ascontiguousarray(j, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        x = np.ascontiguousarray(aj_new, dtype=np.complex128)
        y = np.ascontiguousarray(ak_new, dtype=np.complex128)
        dE = np.zeros(len(j))
        _check(lib().rlpt_pair_dE(self._h, copy, len(j), _ptr(j), _ptr(k), _ptr(x), _ptr(y), _ptr(dE)))
        return dE

    def observables(self) -> dict:
        S, T, B, Lh = self.S, self.T, self.cfg.n_bins, max(self.cfg.series_len, 1)
        shapes = {"hist": (S, T, B), "hist_I": (S, T, B), "spectrum": (S, T, max(self.Ns)),
                  "swap_acc": (S, max(T - 1, 1)), "swap_tries": (S, max(T - 1, 1)),
                  "series_e": (S, T, Lh), "series_q": (S, T, Lh)}
        out = {f: np.zeros(shapes.get(f, (S, T))) for f in OBS_FIELDS}
        o = Obs(**{f: _ptr(out[f]).value for f in OBS_FIELDS})
        _check(lib().rlpt_observables(self._h, C.byref(o)))
        return out


def tune_clear():
    _check(lib().rlpt_tune_clear())


def tune_set(n_modes, precision, shared_pairs, block_threads, copies_per_block, ms_per_sweep):
    t = Tile(n_modes=n_modes, precision=precision, shared_pairs=shared_pairs, block_threads=block_threads,
             copies_per_block=copies_per_block, ms_per_sweep=ms_per_sweep)
    _check(lib().rlpt_tune_set(C.byref(t)))


def tune_entries() -> list:
    n = C.c_int32()
    _check(lib().rlpt_tune_get(None, 0, C.byref(n)))
    arr = (Tile * max(n.value, 1))()
    _check(lib().rlpt_tune_get(arr, n.value, C.byref(n)))
    return [{f: getattr(arr[i], f) for f, _ in Tile._fields_ if f != "pad"} for i in range(n.value)]


def tune_save(path: str):
    _check(lib().rlpt_tune_save(path.encode()))


def tune_load(path: str):
    _check(lib().rlpt_tune_load(path.encode()))


def autotune(graphs, temps, config: Config | None = None, sweeps_per_trial: int = 3, device: str = "cuda:0",
             **kw) -> int:
    """Time every sweep tile for each N among graphs (fills the tile registry); returns trials run."""
    import torch

    cfg = config if config is not None else default_config(**kw)
    temps = np.ascontiguousarray(temps, dtype=np.float64)
    arr = (C.c_void_p * len(graphs))(*[g._h.value for g in graphs])
    nbytes = C.c_size_t()
    _check(lib().rlpt_workspace_size(C.byref(cfg), arr, len(graphs), C.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
    stream = torch.cuda.Stream(device=device)
    n = C.c_int32()
    _check(lib().rlpt_autotune(C.byref(cfg), arr, len(graphs), _ptr(temps), C.c_void_p(ws.data_ptr()), nbytes.value,
                               C.c_void_p(stream.cuda_stream), sweeps_per_trial, C.byref(n)))
    stream.synchronize()
    return n.value


SUMMARY_FIELDS = ["E", "E_err", "cv", "cv_err", "q2", "q2_err", "kurtosis", "kurtosis_err", "y2", "y2_err", "y4",
                  "y4_err", "acc_rate", "swap_rate"]


class Summary(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in SUMMARY_FIELDS]


def summarize(obs: dict, n_modes: int, temps) -> dict:
    """Per-temperature disorder averages and jackknife errors (rlpt_summarize)."""
    temps = np.ascontiguousarray(temps, dtype=np.float64)
    S, T = obs["e_n"].shape
    arrs = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in obs.items()}
    o = Obs(**{f: _ptr(arrs[f]).value for f in OBS_FIELDS if f in arrs})
    out = {f: np.zeros(max(T - 1, 1) if f == "swap_rate" else T) for f in SUMMARY_FIELDS}
    s = Summary(**{f: _ptr(out[f]).value for f in SUMMARY_FIELDS})
    _check(lib().rlpt_summarize(C.byref(o), S, T, n_modes, _ptr(temps), C.byref(s)))
    return out


def adaptive_ladder(T_grid, C_grid, T_min: float, T_max: float, c: float = 0.6, capacity: int = 1024) -> np.ndarray:
    """Temperatures with spacing adapted to the specific heat (rlpt_adaptive_ladder; c is the
    constant C of the rule)."""
    Tg = np.ascontiguousarray(T_grid, dtype=np.float64)
    Cg = np.ascontiguousarray(C_grid, dtype=np.float64)
    out = np.zeros(capacity)
    n = C.c_int32()
    _check(lib().rlpt_adaptive_ladder(_ptr(Tg), _ptr(Cg), len(Tg), T_min, T_max, c, _ptr(out), capacity, C.byref(n)))
    return out[:n.value].copy()


def window_means(x, capacity: int = 64):
    """Means over doubling windows [0,1), [1,2), [2,4), ... and their starts."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = np.zeros(capacity)
    st = np.zeros(capacity, dtype=np.int64)
    n = C.c_int32()
    _check(lib().rlpt_window_means(_ptr(x), len(x), _ptr(m), _ptr(st), capacity, C.byref(n)))
    return m[:n.value].copy(), st[:n.value].copy()


def tau_int(x, c_window: float = 6.0):
    """Integrated autocorrelation time (Sokal's automatic window); returns (tau, window)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    tau, W = C.c_double(), C.c_int64()
    _check(lib().rlpt_tau_int(_ptr(x), len(x), c_window, C.byref(tau), C.byref(W)))
    return tau.value, W.value
