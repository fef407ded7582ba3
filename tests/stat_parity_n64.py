"""Statistical parity of the N = 64 configuration (8 samples x 24 temperatures
geometric in [0.3, 1.5] x 2 replicas, FP32 fields with FP64 recomputation every
100 sweeps) against the FP64 CPU oracle run in full on the same disorder and
seeds, as independent chains once FP32 rounding has separated them.

Not collected by pytest (minutes of oracle time); run on a GPU host:

    python tests/stat_parity_n64.py [sweeps]     # default 10^5, the configuration's length

Prints one JSON line: per temperature and observable (E, C_V, <q^2>, Y_2) the
z-score of the mean over samples of the paired difference (both runs see the
same disorder; jackknife error over samples), the fraction of cells within
2 sigma, the largest z, and sum z^2 beside its expectation (S - 1)/(S - 3) per
cell for a t law with S - 1 degrees of freedom (cells at neighbouring
temperatures are correlated through the swaps, so this is a rough check),
and the collected tests' t-law rule (count within 2 sigma, mean z^2, largest
z against their thresholds).
It also times the oracle: the whole run of the N = 64 configuration, and the
N = 16 FP64 configuration (1 sample x 8 temperatures x 2 replicas, 2000
sweeps) in full.
The same comparison between two GPU runs with different seeds calibrates what
the slow cold end does to such a test at this run length.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2511_13508_amd import rlpt  # noqa: E402
from tests.test_gpu_parity import jackknife, oracle_stack, per_sample_obs, same_law_report  # noqa: E402

N, S, T, REPS = 64, 8, 24, 2
SEED = 2511135080 + 500  # disorder seed of sample mu in the N = 64 configuration: SEED + mu


def gpu_run(graphs, temps, sweeps, run_seed):
    import torch
    ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=REPS, precision=rlpt.FP32, swap_interval=1,
                       resync_interval=100, measure_start=sweeps // 2, measure_interval=1, n_bins=100)
    ctx.init(run_seed)
    ctx.sweep(sweeps)
    torch.cuda.synchronize()
    ctx.check()
    obs = ctx.observables()
    ctx.close()
    return per_sample_obs(obs, temps)


def z_scores(a, b):
    out = {}
    for k in ("E", "C_V", "q2", "Y2"):
        m, s = jackknife(a[k] - b[k])
        out[k] = np.abs(m) / np.maximum(s, 1e-300)
    return out


def summary(z, temps):
    allz = np.concatenate([v for v in z.values()])
    return {"within_2sigma": float(np.mean(allz <= 2.0)), "max_z": float(allz.max()),
            "sum_z2": float(np.sum(allz ** 2)), "sum_z2_expected_t_law": allz.size * (S - 1) / (S - 3),
            "z_by_observable": {k: np.round(v, 2).tolist() for k, v in z.items()},
            "within_2sigma_T_ge_0.6": float(np.mean(np.concatenate([v[temps >= 0.6] for v in z.values()]) <= 2.0))}


def main():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    sweeps = int(sys.argv[1]) if len(sys.argv) > 1 else 100000
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    graphs = [rlpt.Graph(N, SEED + mu) for mu in range(S)]
    g1 = gpu_run(graphs, temps, sweeps, 1)
    g2 = gpu_run(graphs, temps, sweeps, 2)
    t0 = time.perf_counter()
    ors = []
    for mu in range(S):
        pt = O.PT(O.Graph(N, SEED + mu), temps, n_reps=REPS, run_seed=1, sample=mu, swap_interval=1,
                  resync_interval=100, measure_start=sweeps // 2, measure_interval=1, n_bins=100)
        pt.run(sweeps)
        ors.append(pt)
        print(f"oracle sample {mu} done ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    o_sec = time.perf_counter() - t0
    o = per_sample_obs(oracle_stack(ors), temps)
    t16 = 0.3 * (1.5 / 0.3) ** (np.arange(8) / 7)
    t0 = time.perf_counter()
    O.PT(O.Graph(16, 2511135080), t16, n_reps=2, run_seed=1, swap_interval=1, measure_start=1000).run(2000)
    o16_sec = time.perf_counter() - t0
    print(json.dumps({"config": f"N={N}, {S} samples x {T} T [0.3, 1.5] x {REPS} replicas, {sweeps} sweeps, "
                                f"second half measured",
                      "oracle": {"seconds": o_sec, "threads": int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count(),
                                 "mode_updates_per_s": S * T * REPS * N * sweeps / o_sec,
                                 "n16_fp64_full_run_seconds": o16_sec},
                      "gpu_vs_oracle": summary(z_scores(g1, o), temps),
                      "gpu_vs_gpu_other_seed": summary(z_scores(g1, g2), temps),
                      "t_law_rule": {name: {k: v for k, v in same_law_report(a, b, ("E", "C_V", "q2", "Y2")).items()
                                            if k != "z"}
                                     for name, (a, b) in (("gpu_vs_oracle", (g1, o)), ("gpu_vs_gpu", (g1, g2)))}}),
          flush=True)


if __name__ == "__main__":
    main()
