"""GPU parity on sparse mode-locked graphs (finite connectivity per mode,
c = floor(z N / 4) matched terms) against the CPU FP64 oracle on the same
graphs: FP64 trajectories bit-for-bit in every discrete decision, FP32 in
law."""
import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests.gpu_util import make_ctx, oracle_pt
from tests.test_gpu_parity import SEED0, assert_same_law, compare_fp64, temps_geo

pytestmark = pytest.mark.gpu


def run_sparse(oracle, Ns, z, temps, n_sweeps, seed, oracle_seed=None, **cfg):
    seeds = [SEED0 + 500 + i for i in range(len(Ns))]
    graphs = [rlpt.Graph(N, s, mean_degree=z) for N, s in zip(Ns, seeds)]
    ctx = make_ctx(graphs, temps, n_temps=len(temps), **cfg)
    ctx.init(seed)
    ctx.sweep(n_sweeps)
    ctx.check()
    ors = []
    for mu, (N, s) in enumerate(zip(Ns, seeds)):
        pt = oracle_pt(oracle, oracle.Graph(N, s, mean_degree=z), temps, mu, ctx.cfg,
                       seed if oracle_seed is None else oracle_seed, shared_pairs=bool(ctx.cfg.shared_pairs))
        pt.run(n_sweeps)
        ors.append(pt)
    return ctx, ors


@pytest.mark.parametrize("field_mode", [rlpt.FIELDS_STREAM, rlpt.FIELDS_CACHED])
def test_sparse_trajectory_fp64_n256(oracle, field_mode):
    """N = 256, mean degree 16 (1024 terms), 8 temperatures, 2 replicas, 300 sweeps."""
    ctx, ors = run_sparse(oracle, [256], 16, temps_geo(0.3, 1.5, 8), 300, 3, n_reps=2, precision=rlpt.FP64,
                          resync_interval=50, measure_start=100, n_bins=20, field_mode=field_mode)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("shared", [0, 1])
def test_sparse_trajectory_fp64_n1024(oracle, shared):
    """N = 1024 (the largest index width), mean degree 32 (8192 terms)."""
    ctx, ors = run_sparse(oracle, [1024], 32, temps_geo(0.3, 1.5, 4), 40, 4, n_reps=2, precision=rlpt.FP64,
                          shared_pairs=shared, resync_interval=20, n_bins=10)
    compare_fp64(ctx, ors)


def test_sparse_uneven_batch_fp64(oracle):
    ctx, ors = run_sparse(oracle, [512, 128, 1000, 64], 12, temps_geo(0.4, 1.5, 3), 30, 5, n_reps=2,
                          precision=rlpt.FP64, resync_interval=10, n_bins=10)
    compare_fp64(ctx, ors)


def test_sparse_statistical_parity_fp32(oracle):
    """FP32 PT on sparse N = 128 graphs (mean degree 12) and the FP64 oracle as
    independent chains: 12 samples, 8 temperatures, 2 replicas, 4000 sweeps."""
    temps = temps_geo(0.3, 1.5, 8)
    ctx, ors = run_sparse(oracle, [128] * 12, 12, temps, 4000, 51, oracle_seed=1051, n_reps=2,
                          precision=rlpt.FP32, swap_interval=1, resync_interval=100, measure_start=2000,
                          measure_interval=1, n_bins=50)
    assert_same_law(ctx, ors, temps)
