"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
identical seeded inputs.

Tolerances (readings of "1e-5 relative in FP32" for quantities that can
cancel):
  * fields: |F_gpu - F_ora| <= 1e-5 * max(|F_ora|, rms_l |F_ora|)  (FP32),
    1e-12 (FP64);
  * pair dE: |dE_gpu - dE_ora| <= 1e-5 * 2 (|d_j||F_j| + |d_k||F_k|), the
    magnitude before cancellation (FP32); 1e-12 (FP64);
  * FP64 energy recomputation: 1e-10 relative;
  * FP64 trajectories: states 1e-9, integer results (temperatures,
    acceptance and swap counts, histograms) exact.
"""
import math

import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests import synth
from tests.gpu_util import assert_fields_close, make_ctx, oracle_pt, random_states, rounded

pytestmark = pytest.mark.gpu

SEED0 = 2511135080  # disorder seeds: SEED0 + 100 * config + sample


def temps_geo(lo, hi, n):
    return synth.geometric_temps(lo, hi, n)


# ------------------------------------------------------------------ init
@pytest.mark.parametrize("precision", [rlpt.FP64, rlpt.FP32])
def test_init_matches_oracle(oracle, precision):
    Ns = [16, 24]
    graphs = [rlpt.Graph(N, SEED0 + i) for i, N in enumerate(Ns)]
    ctx = make_ctx(graphs, temps_geo(0.3, 1.5, 4), n_temps=4, n_reps=2, precision=precision)
    ctx.init(77)
    a = ctx.get_state()
    E, temp_of = ctx.energies()
    off = 0
    tol = 1e-12 if precision == rlpt.FP64 else 3e-7
    for c in range(ctx.n_copies):
        N = Ns[c // ctx.R]
        ref = oracle.init_copy(N, 77, c)
        np.testing.assert_allclose(a[off:off + N], ref, rtol=0, atol=tol * 2)
        og = oracle.Graph(N, SEED0 + c // ctx.R)
        assert E[c] == pytest.approx(oracle.energy(og, rounded(a[off:off + N], precision)), rel=1e-6, abs=1e-6)
        off += N
    assert np.array_equal(temp_of, np.tile(np.arange(4), 2 * len(Ns)))


# ------------------------------------------------------------------ fields / pair dE / energy
PK, CH = rlpt.LAYOUT_PACKED, rlpt.LAYOUT_CHUNKED
CASES = [(16, rlpt.FP64, PK), (16, rlpt.FP32, PK), (16, rlpt.FP32, CH), (64, rlpt.FP32, PK), (64, rlpt.FP32, CH),
         (97, rlpt.FP32, CH), (97, rlpt.FP32, PK), (64, rlpt.FP64, CH), (256, rlpt.FP32, CH)]


@pytest.mark.parametrize("N,precision,layout", CASES)
def test_local_fields_match_oracle(oracle, N, precision, layout):
    g = rlpt.Graph(N, SEED0 + N)
    og = oracle.Graph(N, SEED0 + N)
    ctx = make_ctx([g], temps_geo(0.3, 1.5, 2), n_temps=2, n_reps=2, precision=precision, list_layout=layout)
    ctx.init(1)
    states = synth.random_state(N, 5, n_copies=ctx.n_copies)
    ctx.set_state(states)
    rel = 1e-12 if precision == rlpt.FP64 else 1e-5
    n_floor = 0
    for c in range(ctx.n_copies):
        F = ctx.local_fields(c)
        ref = oracle.fields(og, rounded(states[c], precision))
        n_floor += assert_fields_close(F, ref, rel)
    print(f"N={N}: {n_floor} of {N * ctx.n_copies} modes within the rms floor but not within {rel} of their own |F|")


@pytest.mark.parametrize("N,precision,layout", CASES)
def test_pair_dE_matches_oracle(oracle, N, precision, layout):
    g = rlpt.Graph(N, SEED0 + N)
    og = oracle.Graph(N, SEED0 + N)
    ctx = make_ctx([g], [1.0], n_temps=1, n_reps=1, precision=precision, list_layout=layout)
    ctx.init(2)
    a = synth.random_state(N, 6)
    ctx.set_state(a)
    ar = rounded(a, precision)
    pairs = synth.random_pairs(N, 7, 24 if N < 200 else 6)
    new = rounded(synth.random_complex(8, 2 * len(pairs)), precision)
    dE = ctx.pair_dE(0, pairs[:, 0], pairs[:, 1], new[0::2], new[1::2])
    F = oracle.fields(og, ar)
    for p, (j, k) in enumerate(pairs):
        ref = oracle.pair_dE(og, ar, int(j), int(k), new[2 * p], new[2 * p + 1])
        if precision == rlpt.FP64:
            tol = 1e-12 * max(1.0, abs(ref))
        else:
            b = ar.copy()
            b[j] = new[2 * p]
            Fk = oracle.fields(og, b)[k]
            tol = 1e-5 * 2 * (abs(new[2 * p] - ar[j]) * abs(F[j]) + abs(new[2 * p + 1] - ar[k]) * abs(Fk))
        assert abs(dE[p] - ref) <= tol, (p, dE[p], ref, tol)


@pytest.mark.parametrize("N,precision,layout", CASES)
def test_energy_fp64_matches_oracle(oracle, N, precision, layout):
    g = rlpt.Graph(N, SEED0 + N)
    og = oracle.Graph(N, SEED0 + N)
    ctx = make_ctx([g], temps_geo(0.5, 1.0, 3), n_temps=3, n_reps=2, precision=precision, list_layout=layout)
    ctx.init(3)
    states = synth.random_state(N, 9, n_copies=ctx.n_copies)
    ctx.set_state(states)
    E = ctx.energy_fp64()
    for c in range(ctx.n_copies):
        ref = oracle.energy(og, rounded(states[c], precision))
        assert E[c] == pytest.approx(ref, rel=1e-10, abs=1e-12)


# ------------------------------------------------------------------ trajectories
def run_pair(oracle, Ns, temps, n_sweeps, seed, seeds=None, omega=rlpt.OMEGA_RANDOM, oracle_shared=None,
             oracle_seed=None, **cfg):
    seeds = seeds or [SEED0 + i for i in range(len(Ns))]
    graphs = [rlpt.Graph(N, s, omega) for N, s in zip(Ns, seeds)]
    ctx = make_ctx(graphs, temps, n_temps=len(temps), **cfg)
    ctx.init(seed)
    ctx.sweep(n_sweeps)
    ctx.check()
    ors = []
    for mu, (N, s) in enumerate(zip(Ns, seeds)):
        kw = {} if oracle_shared is None else {"shared_pairs": oracle_shared}
        pt = oracle_pt(oracle, oracle.Graph(N, s, omega), temps, mu, ctx.cfg,
                       seed if oracle_seed is None else oracle_seed, **kw)
        pt.run(n_sweeps)
        ors.append(pt)
    return ctx, ors


def compare_fp64(ctx, ors, state_tol=1e-9):
    a = ctx.get_state()
    E, temp_of = ctx.energies()
    obs = ctx.observables()
    off = 0
    for mu, pt in enumerate(ors):
        N = pt.g.N
        R = ctx.R
        np.testing.assert_allclose(a[off:off + R * N], pt.a.ravel(), rtol=0, atol=state_tol)
        off += R * N
        np.testing.assert_allclose(E[mu * R:(mu + 1) * R], pt.E, rtol=1e-9, atol=1e-9)
        assert np.array_equal(temp_of[mu * R:(mu + 1) * R], pt.temp_of)
        A = pt.acc
        assert np.array_equal(obs["acc"][mu], A["acc"])
        assert np.array_equal(obs["tries"][mu], A["tries"])
        if ctx.T > 1:
            assert np.array_equal(obs["swap_acc"][mu], A["swap_acc"])
            assert np.array_equal(obs["swap_tries"][mu], A["swap_tries"])
        for f in ("e_n", "q_n"):
            assert np.array_equal(obs[f][mu], A[f])
        for f in ("e_sum", "e_sq", "y2_sum", "y4_sum", "q_sum", "q_sq", "q_4"):
            np.testing.assert_allclose(obs[f][mu], A[f], rtol=1e-9, atol=1e-9)
        assert np.array_equal(obs["hist"][mu], A["hist"])
        assert np.array_equal(obs["hist_I"][mu], A["hist_I"])
        np.testing.assert_allclose(obs["spectrum"][mu][:, :N], A["spectrum"], rtol=1e-9, atol=1e-9)
        assert not np.any(obs["spectrum"][mu][:, N:])


@pytest.mark.parametrize("layout", [PK, CH])
def test_trajectory_fp64_config0(oracle, layout):
    """Plain PT in FP64 at N = 16, 8 temperatures geometric in [0.3, 1.5], two
    replicas, 2000 sweeps, a swap round every sweep: the whole run, bit-for-bit
    in every discrete decision."""
    ctx, ors = run_pair(oracle, [16], temps_geo(0.3, 1.5, 8), 2000, 11, seeds=[SEED0], n_reps=2,
                        precision=rlpt.FP64, swap_interval=1, resync_interval=100, measure_start=1000,
                        measure_interval=1, n_bins=100, series_len=64, list_layout=layout)
    compare_fp64(ctx, ors)
    obs = ctx.observables()
    np.testing.assert_allclose(obs["series_e"][0], ors[0].acc["series_e"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(obs["series_q"][0], ors[0].acc["series_q"], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("shared,layout", [(0, PK), (1, PK), (0, CH), (1, CH)])
def test_trajectory_fp64_uneven_batch(oracle, shared, layout):
    """Several samples of different N in one launch, both pair schedules."""
    ctx, ors = run_pair(oracle, [24, 16, 33, 12], temps_geo(0.4, 1.5, 5), 150, 5, n_reps=2,
                        precision=rlpt.FP64, shared_pairs=shared, swap_interval=2, resync_interval=30,
                        measure_start=50, measure_interval=3, n_bins=20, list_layout=layout)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("block,copies", [(64, 1), (128, 1), (256, 2), (512, 4), (256, 4)])
def test_trajectory_fp64_tiles(oracle, block, copies):
    """Every launch tile gives the same trajectory."""
    ctx, ors = run_pair(oracle, [20], temps_geo(0.5, 1.2, 3), 60, 9, n_reps=3, precision=rlpt.FP64,
                        block_threads=block, copies_per_block=copies, resync_interval=0, n_bins=10)
    compare_fp64(ctx, ors)


@pytest.mark.parametrize("N,block,copies", [(20, 256, 1), (64, 256, 1), (128, 512, 1), (128, 512, 2),
                                            (20, 256, 4), (32, 256, 4), (48, 256, 4)])
def test_trajectory_fp64_chunks_a_step_ahead(oracle, N, block, copies):
    """Chunked lists held in registers ahead of their step.  With one copy per
    workgroup each list goes to half of the copy's waves when it still fits:
    at most 35 chunks per list at N = 20 (1 per thread of 128) and 357 at
    N = 64 (3 per thread of 128, the 4-chunk variant); 1428 at N = 128 would
    need 6 per thread of 256, so both lists go to all 512 threads (3 each,
    the 4-chunk variant); two copies per 512-thread workgroup need 6 per thread
    and stream instead.  Four copies per 256-thread workgroup leave one wave
    per copy, which cannot be halved: N = 20, 32 and 48 then hold 1, 2 and 3
    chunks per thread of 64 (the 1-, 2- and 4-chunk variants).  Every one
    gives the oracle's trajectory."""
    ctx, ors = run_pair(oracle, [N], temps_geo(0.5, 1.2, 3), 20, 13, n_reps=2, precision=rlpt.FP64,
                        block_threads=block, copies_per_block=copies, resync_interval=0, n_bins=10,
                        list_layout=CH)
    compare_fp64(ctx, ors)


def test_edge_cases_fp64(oracle):
    """N = 4 comb (one term), odd N = 5, a single temperature and one replica."""
    for N, omega in ((4, rlpt.OMEGA_COMB), (5, rlpt.OMEGA_COMB), (7, rlpt.OMEGA_RANDOM)):
        ctx, ors = run_pair(oracle, [N], [0.7], 300, 3, seeds=[SEED0 + 9], omega=omega, n_reps=1,
                            precision=rlpt.FP64, resync_interval=50, n_bins=8)
        compare_fp64(ctx, ors)


@pytest.mark.parametrize("layout", [PK, CH])
def test_trajectory_fp32_until_first_flip(oracle, layout):
    """FP32 fields: the same discrete decisions as the FP64 oracle over a short
    run; states agree to FP32 accuracy.  A boundary flip (a uniform within
    FP32 rounding of the acceptance threshold) may separate at most one copy."""
    ctx, ors = run_pair(oracle, [64], temps_geo(0.3, 1.5, 8), 3, 21, n_reps=2, precision=rlpt.FP32,
                        resync_interval=0, n_bins=10, list_layout=layout)
    a = ctx.get_state().reshape(ctx.R, 64)
    E, temp_of = ctx.energies()
    bad = 0
    for c in range(ctx.R):
        ok = np.allclose(a[c], ors[0].a[c], rtol=0, atol=2e-5) and temp_of[c] == ors[0].temp_of[c]
        ok = ok and abs(E[c] - ors[0].E[c]) <= 1e-4 * max(1.0, abs(ors[0].E[c]))
        bad += 0 if ok else 1
    assert bad <= 1, bad


def test_graph_replay_is_bitwise_equal_to_plain_sweeps():
    graphs = [rlpt.Graph(32, SEED0 + 1), rlpt.Graph(32, SEED0 + 2)]
    temps = temps_geo(0.3, 1.5, 6)
    kw = dict(n_temps=6, n_reps=2, precision=rlpt.FP32, swap_interval=2, resync_interval=10, measure_start=0,
              measure_interval=1, n_bins=16, series_len=40)
    c1 = make_ctx(graphs, temps, **kw)
    c2 = make_ctx(graphs, temps, **kw)
    c1.init(4)
    c2.init(4)
    c1.sweep(40)
    for _ in range(3):  # replays after a re-capture with the same key
        c2.run_graph(10, 1)
    c2.run_graph(10, 1)
    assert np.array_equal(c1.get_state(), c2.get_state())
    o1, o2 = c1.observables(), c2.observables()
    for f in o1:
        assert np.array_equal(o1[f], o2[f]), f
    assert c1.counters() == c2.counters()


def test_run_twice_is_deterministic():
    g = [rlpt.Graph(48, SEED0 + 3)]
    out = []
    for _ in range(2):
        ctx = make_ctx(g, temps_geo(0.3, 1.5, 8), n_temps=8, n_reps=2, precision=rlpt.FP32)
        ctx.init(6)
        ctx.sweep(25)
        out.append((ctx.get_state(), ctx.energies()[0]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


# ------------------------------------------------------------------ recomputation and failure handling
def test_resync_restores_constraint_and_energy(oracle):
    N = 32
    g = rlpt.Graph(N, SEED0 + 5)
    og = oracle.Graph(N, SEED0 + 5)
    ctx = make_ctx([g], [0.5, 1.0], n_temps=2, n_reps=1, precision=rlpt.FP32, drift_tol=0.0)
    ctx.init(8)
    a = ctx.get_state().reshape(2, N) * 1.01  # off the constraint surface by ~4%
    ctx.set_state(a)
    ctx.resync()
    b = ctx.get_state().reshape(2, N)
    E, _ = ctx.energies()
    for c in range(2):
        assert np.sum(np.abs(b[c]) ** 4) == pytest.approx(N, rel=3e-6)
        assert E[c] == pytest.approx(oracle.energy(og, rounded(b[c], rlpt.FP32)), rel=1e-5)


def test_drift_is_reported_as_state_error(tmp_path):
    """Changing the state behind the running energy is caught at the next
    recomputation (host-forced condition; every kernel exits normally).  The
    state is changed in a checkpoint file, whose first region holds the FP32
    amplitudes after an 80-byte header and an 8-byte region length, and
    loaded back with its old running energies; set_state, by contrast,
    recomputes the energies of the configuration it writes."""
    g = rlpt.Graph(16, SEED0 + 6)
    ctx = make_ctx([g], [1.0], n_temps=1, n_reps=2, precision=rlpt.FP32, resync_interval=5, drift_tol=1e-3)
    ctx.init(1)
    ctx.set_state(np.conj(ctx.get_state()[::-1]).copy())  # a new configuration with its own energy: no drift
    ctx.sweep(5)
    ctx.check()
    path = str(tmp_path / "ck.bin")
    ctx.checkpoint_save(path)
    raw = bytearray(open(path, "rb").read())
    n = int(np.frombuffer(bytes(raw[80:88]), dtype=np.uint64)[0])
    assert n == 2 * 16 * 2 * 4
    amp = np.frombuffer(bytes(raw[88:88 + n]), dtype=np.complex64)
    raw[88:88 + n] = np.conj(amp[::-1]).astype(np.complex64).tobytes()  # different configuration, stale energy
    open(path, "wb").write(bytes(raw))
    ctx.checkpoint_load(path)
    ctx.sweep(5)
    with pytest.raises(rlpt.RlptError) as e:
        ctx.check()
    assert e.value.code == rlpt.RLPT_E_STATE


def test_set_state_sets_the_running_energies(oracle):
    """set_state recomputes every copy's running energy from the configuration it writes."""
    N = 24
    g = rlpt.Graph(N, SEED0 + 7)
    og = oracle.Graph(N, SEED0 + 7)
    ctx = make_ctx([g], [0.5, 1.0], n_temps=2, n_reps=1, precision=rlpt.FP64, drift_tol=1e-12)
    ctx.init(2)
    a = synth.random_constrained_state(N, 17, 2)
    ctx.set_state(a)
    E, _ = ctx.energies()
    for c in range(2):
        assert E[c] == pytest.approx(oracle.energy(og, a[c]), rel=1e-12, abs=1e-12)
    assert ctx.resync() < 1e-12


def test_set_state_rejects_nan():
    g = rlpt.Graph(8, SEED0)
    ctx = make_ctx([g], [1.0], n_temps=1, n_reps=1)
    ctx.init(1)
    a = ctx.get_state()
    a[0] = np.nan
    with pytest.raises(rlpt.RlptError):
        ctx.set_state(a)


# ------------------------------------------------------------------ statistical parity
def per_sample_obs(A, temps):
    """Per-(sample, T) thermal averages from accumulators with leading sample axis."""
    E = A["e_sum"] / A["e_n"]
    cv = (A["e_sq"] / A["e_n"] - E ** 2) / temps ** 2
    return {"E": E, "C_V": cv, "q2": A["q_sq"] / A["q_n"], "Y2": A["y2_sum"] / A["e_n"], "Y4": A["y4_sum"] / A["e_n"]}


def jackknife(v):
    n = v.shape[0]
    loo = (v.sum(axis=0) - v) / (n - 1)
    return v.mean(axis=0), np.sqrt((n - 1) / n * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))


def oracle_stack(ors):
    keys = ("e_n", "e_sum", "e_sq", "y2_sum", "y4_sum", "q_n", "q_sum", "q_sq", "q_4")
    return {k: np.stack([pt.acc[k] for pt in ors]) for k in keys}


def same_law_report(a, b, keys=("E", "C_V", "q2", "Y2", "Y4")):
    """z per (observable, temperature) cell of the paired differences a - b
    over S disorder samples (jackknife error), with the rule's thresholds.
    Under equal laws z follows a t law with nu = S - 1 degrees of freedom:
    P(z <= 2) = p2, E z^2 = nu / (nu - 2), Var z^2 = 2 nu^2 (nu - 1) / ((nu - 2)^2 (nu - 4))."""
    from scipy import stats
    zs = []
    for k in keys:
        m, s = jackknife(a[k] - b[k])
        s = np.maximum(s, 1e-12 * np.abs(b[k]).mean())
        zs.append(np.abs(m) / s)
    z = np.concatenate(zs)
    S, M = a[keys[0]].shape[0], z.size
    nu = S - 1
    p2 = 2 * stats.t.cdf(2.0, nu) - 1
    ez2 = nu / (nu - 2)
    vz2 = 2 * nu ** 2 * (nu - 1) / ((nu - 2) ** 2 * (nu - 4))
    return {"z": {k: np.round(v, 2) for k, v in zip(keys, zs)}, "cells": M,
            "within_2sigma": int(np.sum(z <= 2)), "within_2sigma_min": M * p2 - 2.5 * np.sqrt(M * p2 * (1 - p2)),
            "mean_z2": float(np.mean(z ** 2)), "mean_z2_max": ez2 + 3 * np.sqrt(vz2 / M),
            "max_z": float(z.max()), "max_z_allowed": float(stats.t.ppf(1 - 0.005 / M, nu))}


def assert_same_law(ctx, ors, temps, keys=("E", "C_V", "q2", "Y2", "Y4")):
    """Per temperature, the disorder averages of <E>, C_V, <q^2>, <Y_2>, <Y_4>
    from two independent runs agree ("within 2 sigma"; the paper gives no
    rule): the paired z of each cell follows a t law with S - 1 degrees of
    freedom, so (1) the count of cells with z <= 2 is at least its t-law
    expectation less 2.5 binomial standard deviations, (2) the mean of z^2
    over cells is at most its expectation (S-1)/(S-3) plus 3 standard errors
    (a shift of every cell by ~1.5 sigma fails it), (3) no z exceeds the
    t quantile of a 1 % family-wise two-sided level."""
    g = per_sample_obs(ctx.observables(), temps)
    o = per_sample_obs(oracle_stack(ors), temps)
    check_same_law(same_law_report(g, o, keys))


def check_same_law(r):
    assert r["within_2sigma"] >= r["within_2sigma_min"], r
    assert r["mean_z2"] <= r["mean_z2_max"], r
    assert r["max_z"] <= r["max_z_allowed"], r


@pytest.mark.parametrize("shared", [0, 1])
def test_statistical_parity_fp32(oracle, shared):
    """FP32 PT on the GPU against the FP64 oracle as two independent chains
    (different run seeds, same disorder): N = 32, 12 disorder samples, 8
    temperatures geometric in [0.3, 1.5], 2 replicas, 4000 sweeps measured
    over the second half.  With the same run seed the FP32 chain follows the
    oracle's decision for decision for thousands of sweeps, and the paired
    differences would then measure only FP32 rounding of the running energy,
    not the law sampled.  With shared pairs the GPU also follows a different
    pair schedule: a check that the shared schedule samples the same law."""
    Ns = [32] * 12
    temps = temps_geo(0.3, 1.5, 8)
    ctx, ors = run_pair(oracle, Ns, temps, 4000, 31, n_reps=2, precision=rlpt.FP32, shared_pairs=shared,
                        swap_interval=1, resync_interval=100, measure_start=2000, measure_interval=1, n_bins=50,
                        oracle_shared=False, oracle_seed=1031)
    assert_same_law(ctx, ors, temps)
