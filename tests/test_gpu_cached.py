"""GPU parity of the cached-field sweep (field_mode = FIELDS_CACHED) against
the CPU FP64 oracle.

The cached sweep keeps every copy's local fields in LDS / HBM and updates
them on acceptance instead of recomputing F_j, F_k from the lists at every
two-mode update.  It runs the same chain on the same draws as the streaming
sweep (sec. III.A), so the oracle's trajectories are the reference; the
fields are updated by fixed-order gathers, so agreement is up to rounding order:
FP64 states within 1e-9 and every discrete decision exact, as for the
streaming path.
"""
import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests.gpu_util import make_ctx, oracle_pt
from tests.test_gpu_parity import SEED0, assert_same_law, compare_fp64, run_pair, temps_geo

pytestmark = pytest.mark.gpu

PK, CH = rlpt.LAYOUT_PACKED, rlpt.LAYOUT_CHUNKED
CACHED = dict(field_mode=rlpt.FIELDS_CACHED)


@pytest.mark.parametrize("layout", [PK, CH])
def test_cached_trajectory_fp64_config0(oracle, layout):
    """N = 16, 8 temperatures geometric in [0.3, 1.5], two replicas, 2000
    sweeps with a swap round every sweep and measurements over the second half."""
    ctx, ors = run_pair(oracle, [16], temps_geo(0.3, 1.5, 8), 2000, 11, seeds=[SEED0], n_reps=2,
                        precision=rlpt.FP64, swap_interval=1, resync_interval=100, measure_start=1000,
                        measure_interval=1, n_bins=100, series_len=64, list_layout=layout, **CACHED)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("layout", [PK, CH])
def test_cached_fields_without_recomputation(oracle, layout):
    """No recomputation at all for 1500 sweeps: the incrementally updated fields
    alone drive the chain (N = 33, odd, so one mode sits out every sweep)."""
    ctx, ors = run_pair(oracle, [33], temps_geo(0.3, 1.5, 4), 1500, 13, n_reps=2, precision=rlpt.FP64,
                        resync_interval=0, n_bins=10, list_layout=layout, **CACHED)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("shared,layout", [(0, PK), (1, PK), (0, CH), (1, CH)])
def test_cached_uneven_batch(oracle, shared, layout):
    """Several samples of different N in one launch, both pair schedules."""
    ctx, ors = run_pair(oracle, [24, 16, 33, 12], temps_geo(0.4, 1.5, 5), 150, 5, n_reps=2,
                        precision=rlpt.FP64, shared_pairs=shared, swap_interval=2, resync_interval=30,
                        measure_start=50, measure_interval=3, n_bins=20, list_layout=layout, **CACHED)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("block,copies", [(64, 1), (128, 1), (256, 2), (512, 4), (256, 4), (512, 1), (1024, 1)])
def test_cached_tiles(oracle, block, copies):
    """Every launch tile gives the same trajectory."""
    ctx, ors = run_pair(oracle, [20], temps_geo(0.5, 1.2, 3), 60, 9, n_reps=3, precision=rlpt.FP64,
                        block_threads=block, copies_per_block=copies, resync_interval=0, n_bins=10, **CACHED)
    compare_fp64(ctx, ors)


def test_cached_edge_cases(oracle):
    """N = 4 comb (one term), N = 5 comb, N = 7 random: one temperature, one replica."""
    for N, omega in ((4, rlpt.OMEGA_COMB), (5, rlpt.OMEGA_COMB), (7, rlpt.OMEGA_RANDOM)):
        ctx, ors = run_pair(oracle, [N], [0.7], 300, 3, seeds=[SEED0 + 9], omega=omega, n_reps=1,
                            precision=rlpt.FP64, resync_interval=50, n_bins=8, **CACHED)
        compare_fp64(ctx, ors)


def test_cached_fp64_n256(oracle):
    """The headline size N = 256 (chunked lists, 244 pair entries per ordered
    pair on average): 8 temperatures geometric in [0.25, 1.5], 2 replicas,
    20 sweeps against the oracle."""
    ctx, ors = run_pair(oracle, [256], temps_geo(0.25, 1.5, 8), 20, 17, seeds=[SEED0 + 400], n_reps=2,
                        precision=rlpt.FP64, resync_interval=0, n_bins=10, **CACHED)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("layout", [PK, CH])
def test_cached_fp32_until_first_flip(oracle, layout):
    """FP32 cached fields: the same discrete decisions as the FP64 oracle over a
    short run; a boundary flip may separate at most one copy."""
    ctx, ors = run_pair(oracle, [64], temps_geo(0.3, 1.5, 8), 3, 21, n_reps=2, precision=rlpt.FP32,
                        resync_interval=0, n_bins=10, list_layout=layout, **CACHED)
    a = ctx.get_state().reshape(ctx.R, 64)
    E, temp_of = ctx.energies()
    bad = 0
    for c in range(ctx.R):
        ok = np.allclose(a[c], ors[0].a[c], rtol=0, atol=2e-5) and temp_of[c] == ors[0].temp_of[c]
        ok = ok and abs(E[c] - ors[0].E[c]) <= 1e-4 * max(1.0, abs(ors[0].E[c]))
        bad += 0 if ok else 1
    assert bad <= 1, bad


def test_cached_fp32_running_energy_stays_exact():
    """FP32 at N = 256 for 300 sweeps without recomputation: the running energy
    built from cached-field dE stays within 1e-3 relative of the FP64 energy
    of the final state (the default drift tolerance)."""
    g = rlpt.Graph(256, SEED0 + 401)
    ctx = make_ctx([g], temps_geo(0.25, 1.5, 8), n_temps=8, n_reps=2, precision=rlpt.FP32, resync_interval=0,
                   **CACHED)
    ctx.init(3)
    ctx.sweep(300)
    E, _ = ctx.energies()
    E64 = ctx.energy_fp64()
    rel = np.abs(E - E64) / np.maximum(np.abs(E64), 1.0)
    assert rel.max() < 1e-3, rel.max()


def test_cached_statistical_parity_fp32(oracle):
    """FP32 cached PT and the FP64 oracle as independent chains (different run
    seeds): N = 32, 12 samples, 8 temperatures geometric in [0.3, 1.5], 2
    replicas, 4000 sweeps measured over the second half; same law per
    temperature for <E>, C_V, <q^2>, <Y_2>, <Y_4>."""
    Ns = [32] * 12
    temps = temps_geo(0.3, 1.5, 8)
    ctx, ors = run_pair(oracle, Ns, temps, 4000, 37, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                        resync_interval=100, measure_start=2000, measure_interval=1, n_bins=50, oracle_seed=1037,
                        **CACHED)
    assert_same_law(ctx, ors, temps)


def test_cached_fp32_follows_oracle_trajectory(oracle):
    """With the same run seed the FP32 cached chain takes the oracle's
    decisions: N = 32, 8 samples, 8 temperatures, 2 replicas, 1000 sweeps;
    at least 120 of the 128 copies end within 1e-3 of the oracle's state (a
    boundary flip, a uniform within FP32 rounding of its threshold, separates
    a copy for good)."""
    Ns = [32] * 8
    temps = temps_geo(0.3, 1.5, 8)
    ctx, ors = run_pair(oracle, Ns, temps, 1000, 37, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                        resync_interval=100, n_bins=10, **CACHED)
    a = ctx.get_state().reshape(8, 16, 32)
    oa = np.stack([pt.a for pt in ors])
    same = np.all(np.abs(a - oa) < 1e-3, axis=2)
    assert same.sum() >= 120, same.sum()


def test_cached_set_state_refreshes_fields(oracle):
    """After rlpt_set_state the fields are recomputed: a run continued from a
    written state follows the oracle started from the same state."""
    N = 24
    g = rlpt.Graph(N, SEED0 + 402)
    og = oracle.Graph(N, SEED0 + 402)
    temps = temps_geo(0.5, 1.2, 3)
    ctx = make_ctx([g], temps, n_temps=3, n_reps=1, precision=rlpt.FP64, resync_interval=0, n_bins=10,
                   drift_tol=0.0, **CACHED)
    ctx.init(7)
    ctx.sweep(10)
    pt = oracle_pt(oracle, og, temps, 0, ctx.cfg, 7)
    pt.run(10)
    rng = np.random.default_rng(3)
    a = pt.a * np.exp(1j * rng.uniform(0, 2 * np.pi, size=pt.a.shape))  # same |a|: still on the constraint
    ctx.set_state(a.ravel())
    ctx.resync()
    pt.a[:] = a
    for c in range(pt.R):
        pt.E[c] = oracle.energy(og, pt.a[c])
    ctx.sweep(40)
    pt.run(40)
    compare_fp64(ctx, [pt])
