"""Helpers for the GPU parity tests: build matching library / oracle runs."""
from __future__ import annotations

import numpy as np

from paper_2511_13508_amd import rlpt
from tests import synth


def make_ctx(graphs, temps, **cfg):
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return rlpt.Context(graphs, temps, **cfg)


def oracle_pt(oracle, og, temps, sample, ctx_cfg, run_seed, **kw):
    """An oracle PT run mirroring a library context's schedule for one sample."""
    c = ctx_cfg
    kw.setdefault("shared_pairs", bool(c.shared_pairs))
    kw.setdefault("rho", c.rho if c.rho else 4)
    return oracle.PT(og, temps, n_reps=c.n_reps, run_seed=run_seed, sample=sample,
                     swap_interval=c.swap_interval, resync_interval=c.resync_interval, renorm_tol=c.renorm_tol,
                     measure_start=c.measure_start, measure_interval=c.measure_interval, n_bins=c.n_bins,
                     series_len=c.series_len, **kw)


def field_scale(F_ref: np.ndarray) -> float:
    return float(np.sqrt(np.mean(np.abs(F_ref) ** 2)))


def assert_fields_close(F_gpu, F_ref, rel, floor_share=0.02):
    """|F_gpu - F_ref| <= rel * max(|F_ref|, rms(F_ref)) for every mode, and
    at most floor_share of the modes pass only thanks to the rms floor (their
    error exceeds rel * |F_ref|: fields much smaller than typical, where a
    sum of ~N^2 FP32 terms carries the typical field's rounding).  Returns
    that number of modes."""
    s = field_scale(F_ref)
    err = np.abs(F_gpu - F_ref)
    bound = rel * np.maximum(np.abs(F_ref), s)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (bad[:5], err[bad[:5]], bound[bad[:5]])
    n_floor = int(np.sum(err > rel * np.abs(F_ref)))
    assert n_floor <= max(1.0, floor_share * F_ref.size), (n_floor, F_ref.size)
    return n_floor


def rounded(a: np.ndarray, precision: int) -> np.ndarray:
    return a.astype(np.complex64).astype(np.complex128) if precision == rlpt.FP32 else a


def random_states(Ns, R, seed):
    return [synth.random_state(N, seed + i, n_copies=R) for i, N in enumerate(Ns)]
