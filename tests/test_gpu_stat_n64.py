"""GPU: statistical parity of the N = 64 configuration in full size -- 8
disorder samples x 24 temperatures geometric in [0.3, 1.5] x 2 replicas, FP32
fields with FP64 recomputation every 100 sweeps, a swap round every sweep --
against the FP64 CPU oracle on the same disorder, as independent chains
(different run seeds), over 10^4 sweeps with the second half measured (the
configuration runs 10^5; tests/stat_parity_n64.py is that long form).  Per
temperature and observable (E, C_V, <q^2>, Y_2) the paired z over samples
must follow the t law of equal laws (assert_same_law's rule).  Two runs of a
correct chain from the same initial law have the same law at every sweep,
equilibrated or not, so the shortened run tests the same thing."""
import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests.gpu_util import make_ctx
from tests.test_gpu_parity import check_same_law, oracle_stack, per_sample_obs, same_law_report

pytestmark = pytest.mark.gpu

N, S, T, REPS, SWEEPS = 64, 8, 24, 2, 10000
SEED = 2511135080 + 500  # disorder of the N = 64 configuration (as in the long form)


def test_n64_configuration_same_law_as_oracle(oracle):
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    graphs = [rlpt.Graph(N, SEED + mu) for mu in range(S)]
    cfg = dict(n_temps=T, n_reps=REPS, swap_interval=1, resync_interval=100, measure_start=SWEEPS // 2,
               measure_interval=1, n_bins=100)
    ctx = make_ctx(graphs, temps, precision=rlpt.FP32, **cfg)
    ctx.init(11)
    ctx.run_graph(100, SWEEPS // 200)  # HIP-graph segments may not straddle measure_start
    ctx.run_graph(100, SWEEPS // 200)
    ctx.check()
    g = per_sample_obs(ctx.observables(), temps)
    ors = []
    for mu in range(S):
        pt = oracle.PT(oracle.Graph(N, SEED + mu), temps, n_reps=REPS, run_seed=1011, sample=mu, swap_interval=1,
                       resync_interval=100, measure_start=SWEEPS // 2, measure_interval=1, n_bins=100)
        pt.run(SWEEPS)
        ors.append(pt)
    o = per_sample_obs(oracle_stack(ors), temps)
    r = same_law_report(g, o, keys=("E", "C_V", "q2", "Y2"))
    print({k: v for k, v in r.items() if k != "z"})
    check_same_law(r)
