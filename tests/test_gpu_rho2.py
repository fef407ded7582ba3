"""GPU parity of the spherical-constraint variant (rho = 2, sum |a|^2 = N,
the constraint the paper compares the smoothed cubic one with) against the
CPU FP64 oracle run with the same rho.  Same tolerances as the rho = 4
parity tests: FP64 states within 1e-9 and every discrete decision exact."""
import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests.gpu_util import make_ctx, rounded
from tests.test_gpu_parity import SEED0, assert_same_law, compare_fp64, run_pair, temps_geo

pytestmark = pytest.mark.gpu

PK, CH = rlpt.LAYOUT_PACKED, rlpt.LAYOUT_CHUNKED
SPH = dict(rho=2)


@pytest.mark.parametrize("precision", [rlpt.FP64, rlpt.FP32])
def test_rho2_init_matches_oracle(oracle, precision):
    Ns = [16, 24]
    graphs = [rlpt.Graph(N, SEED0 + i) for i, N in enumerate(Ns)]
    ctx = make_ctx(graphs, temps_geo(0.3, 1.5, 4), n_temps=4, n_reps=2, precision=precision, **SPH)
    ctx.init(77)
    a = ctx.get_state()
    off = 0
    tol = 1e-12 if precision == rlpt.FP64 else 3e-7
    for c in range(ctx.n_copies):
        N = Ns[c // ctx.R]
        ref = oracle.init_copy(N, 77, c, rho=2)
        np.testing.assert_allclose(a[off:off + N], ref, rtol=0, atol=tol * 2)
        assert np.sum(np.abs(ref) ** 2) == pytest.approx(N, rel=1e-12)
        off += N


@pytest.mark.parametrize("layout", [PK, CH])
def test_rho2_trajectory_fp64(oracle, layout):
    """N = 16, 8 temperatures geometric in [0.3, 1.5], two replicas, 1500
    sweeps, swaps every sweep, measurements over the second half."""
    ctx, ors = run_pair(oracle, [16], temps_geo(0.3, 1.5, 8), 1500, 12, seeds=[SEED0], n_reps=2,
                        precision=rlpt.FP64, swap_interval=1, resync_interval=100, measure_start=750,
                        measure_interval=1, n_bins=50, series_len=32, list_layout=layout, **SPH)
    compare_fp64(ctx, ors)
    a = ctx.get_state().reshape(ctx.R, 16)
    np.testing.assert_allclose(np.sum(np.abs(a) ** 2, axis=1), 16.0, rtol=1e-12)


@pytest.mark.parametrize("shared", [0, 1])
def test_rho2_uneven_batch_fp64(oracle, shared):
    ctx, ors = run_pair(oracle, [24, 16, 33, 12], temps_geo(0.4, 1.5, 5), 150, 5, n_reps=2,
                        precision=rlpt.FP64, shared_pairs=shared, swap_interval=2, resync_interval=30,
                        measure_start=50, measure_interval=3, n_bins=20, **SPH)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("layout", [PK, CH])
def test_rho2_cached_fields_fp64(oracle, layout):
    """The cached-field sweep with rho = 2 follows the oracle too."""
    ctx, ors = run_pair(oracle, [33], temps_geo(0.3, 1.5, 4), 800, 13, n_reps=2, precision=rlpt.FP64,
                        resync_interval=0, n_bins=10, list_layout=layout, field_mode=rlpt.FIELDS_CACHED, **SPH)
    compare_fp64(ctx, ors)


def test_rho2_fp32_until_first_flip(oracle):
    ctx, ors = run_pair(oracle, [64], temps_geo(0.3, 1.5, 8), 3, 21, n_reps=2, precision=rlpt.FP32,
                        resync_interval=0, n_bins=10, **SPH)
    a = ctx.get_state().reshape(ctx.R, 64)
    E, temp_of = ctx.energies()
    bad = 0
    for c in range(ctx.R):
        ok = np.allclose(a[c], ors[0].a[c], rtol=0, atol=2e-5) and temp_of[c] == ors[0].temp_of[c]
        ok = ok and abs(E[c] - ors[0].E[c]) <= 1e-4 * max(1.0, abs(ors[0].E[c]))
        bad += 0 if ok else 1
    assert bad <= 1, bad


def test_rho2_resync_restores_sphere(oracle):
    N = 32
    g = rlpt.Graph(N, SEED0 + 5)
    og = oracle.Graph(N, SEED0 + 5)
    ctx = make_ctx([g], [0.5, 1.0], n_temps=2, n_reps=1, precision=rlpt.FP32, drift_tol=0.0, **SPH)
    ctx.init(8)
    a = ctx.get_state().reshape(2, N) * 1.02  # off the sphere by ~4%
    ctx.set_state(a)
    ctx.resync()
    b = ctx.get_state().reshape(2, N)
    E, _ = ctx.energies()
    for c in range(2):
        assert np.sum(np.abs(b[c]) ** 2) == pytest.approx(N, rel=3e-6)
        assert E[c] == pytest.approx(oracle.energy(og, rounded(b[c], rlpt.FP32)), rel=1e-5)


def test_rho2_statistical_parity_fp32(oracle):
    """FP32 rho = 2 PT and the FP64 oracle as independent chains: N = 32,
    12 samples, 8 temperatures, 2 replicas, 4000 sweeps."""
    Ns = [32] * 12
    temps = temps_geo(0.3, 1.5, 8)
    ctx, ors = run_pair(oracle, Ns, temps, 4000, 41, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                        resync_interval=100, measure_start=2000, measure_interval=1, n_bins=50, oracle_seed=1041,
                        **SPH)
    assert_same_law(ctx, ors, temps)


def test_rho2_rejects_learned_moves():
    g = rlpt.Graph(16, SEED0)
    with pytest.raises(RuntimeError, match="rho = 4"):
        make_ctx([g], [1.0], n_temps=1, n_reps=2, mlp_nets=1, **SPH)
