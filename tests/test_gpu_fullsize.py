"""GPU parity at full configuration sizes, in the launch configuration the
benchmark times, on sampled disorder samples whose copies the oracle runs in
full over the same sweeps.

* N = 256, 8 samples x 40 temperatures x 2 replicas (640 copies), FP32, the
  chunked lists and built-in tile of the benchmark, both field modes: FP32
  states within 2e-5 of the FP64 oracle; at most one copy per sample may
  separate at an FP32 acceptance-boundary flip.
* N = 64, 8 samples x 24 temperatures x 2 replicas (384 copies) in FP64:
  every discrete decision identical, states within 1e-9.
"""
import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests import synth
from tests.gpu_util import make_ctx, oracle_pt

pytestmark = pytest.mark.gpu

SEED = 2511135080


def fp32_sampled(oracle, ctx, Ns, seeds, temps, sampled, n_sweeps, run_seed):
    a = ctx.get_state()
    E, temp_of = ctx.energies()
    offs = np.concatenate([[0], np.cumsum([ctx.R * N for N in Ns])])
    for mu in sampled:
        N = Ns[mu]
        pt = oracle_pt(oracle, oracle.Graph(N, seeds[mu]), temps, mu, ctx.cfg, run_seed)
        pt.run(n_sweeps)
        ga = a[offs[mu]:offs[mu + 1]].reshape(ctx.R, N)
        bad = 0
        for c in range(ctx.R):
            ok = np.allclose(ga[c], pt.a[c], rtol=0, atol=2e-5) and temp_of[mu * ctx.R + c] == pt.temp_of[c]
            ok = ok and abs(E[mu * ctx.R + c] - pt.E[c]) <= 1e-4 * max(1.0, abs(pt.E[c]))
            bad += 0 if ok else 1
        assert bad <= 1, (mu, bad)


@pytest.mark.parametrize("field_mode", [rlpt.FIELDS_STREAM, rlpt.FIELDS_CACHED])
def test_headline_configuration_sampled(oracle, field_mode):
    N, S, T = 256, 8, 40
    seeds = [SEED + 400 + mu for mu in range(S)]
    graphs = [rlpt.Graph(N, s) for s in seeds]
    temps = 0.25 * (1.5 / 0.25) ** (np.arange(T) / (T - 1))
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=2, precision=rlpt.FP32, swap_interval=1, resync_interval=100,
                   measure_start=0, measure_interval=1, n_bins=100, field_mode=field_mode)
    assert ctx.n_copies == 640
    ctx.init(1)
    ctx.sweep(2)
    ctx.check()
    fp32_sampled(oracle, ctx, [N] * S, seeds, temps, sampled=[0, 5], n_sweeps=2, run_seed=1)


def test_n64_configuration_fp64_sampled(oracle):
    N, S, T = 64, 8, 24
    seeds = [SEED + 100 + mu for mu in range(S)]
    graphs = [rlpt.Graph(N, s) for s in seeds]
    temps = synth.geometric_temps(0.3, 1.5, T)
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=2, precision=rlpt.FP64, swap_interval=1, resync_interval=100,
                   measure_start=10, measure_interval=1, n_bins=100)
    assert ctx.n_copies == 384
    ctx.init(2)
    ctx.sweep(30)
    ctx.check()
    a = ctx.get_state()
    E, temp_of = ctx.energies()
    obs = ctx.observables()
    for mu in (0, 6):
        pt = oracle_pt(oracle, oracle.Graph(N, seeds[mu]), temps, mu, ctx.cfg, 2)
        pt.run(30)
        off = mu * ctx.R * N
        np.testing.assert_allclose(a[off:off + ctx.R * N], pt.a.ravel(), rtol=0, atol=1e-9)
        np.testing.assert_allclose(E[mu * ctx.R:(mu + 1) * ctx.R], pt.E, rtol=1e-9, atol=1e-9)
        assert np.array_equal(temp_of[mu * ctx.R:(mu + 1) * ctx.R], pt.temp_of)
        for f in ("acc", "tries", "swap_acc", "swap_tries", "e_n", "hist", "hist_I"):
            assert np.array_equal(obs[f][mu], pt.acc[f]), f
        np.testing.assert_allclose(obs["spectrum"][mu], pt.acc["spectrum"], rtol=1e-9, atol=1e-9)
