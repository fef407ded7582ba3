"""GPU: the learned global proposal against the FP64 reference (oracle/mlp.py)
and the exactness of its Metropolis-Hastings test.

Tolerances: network outputs 2e-3 relative to their rms (FP32 accumulation vs
FP64); gradients per tensor |g_gpu - g_ora| <= 1e-2 |g_ora| (norms) and
cosine >= 0.999 (the reference is evaluated on the same bfloat16 weights);
proposals 2e-4 absolute; log acceptance ratios 2e-3 absolute (FP32 sums of
~4N log-density terms and of the energy change)."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2511_13508_amd import rlpt
from tests import brute, synth
from tests.gpu_util import make_ctx
from tests.test_gpu_parity import jackknife, oracle_stack, per_sample_obs

pytestmark = pytest.mark.gpu

SEED3 = 2511135080 + 300


def unflatten(p, N, H, K):
    In, D, Out = M.sizes(N, K)
    shapes = [("W1", (In, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, Out)), ("b3", (Out,))]
    out, o = {}, 0
    for k, s in shapes:
        n = int(np.prod(s))
        out[k] = np.asarray(p[o:o + n], dtype=np.float64).reshape(s)
        o += n
    assert o == len(p)
    return out


def mlp_ctx(N, S, T, reps, H, K, batch, nets=2, cap=64, graphs=None, temps=None):
    graphs = graphs or [rlpt.Graph(N, SEED3 + i) for i in range(S)]
    temps = synth.geometric_temps(0.5, 1.5, T) if temps is None else temps
    return make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=nets, mlp_hidden=H,
                    mlp_components=K, mlp_capacity=cap, mlp_batch=batch, resync_interval=0,
                    drift_tol=0.0)


def test_mlp_forward_and_gradients_match_oracle():
    N, H, K, B = 8, 48, 3, 16
    ctx = mlp_ctx(N, 1, 2, 1, H, K, B)
    ctx.init(1)
    ctx.mlp_setup([0, 1], seed=3)
    NP, Out = ctx.mlp_sizes()
    for net in (0, 1):
        p = synth.random_mlp_params(2 * N, H, Out, seed=10 + net, out_scale=0.5)
        assert p.size == NP
        ctx.mlp_set_params(net, p)
        before = synth.random_constrained_state(N, 20 + net, B)
        after = synth.random_constrained_state(N, 30 + net, B)
        ctx.mlp_set_pairs(net, before, after)
    for net in (0, 1):
        params = M.rounded(unflatten(synth.random_mlp_params(2 * N, H, Out, seed=10 + net, out_scale=0.5), N, H, K))
        b = synth.random_constrained_state(N, 20 + net, B).astype(np.complex64).astype(np.complex128)
        a = synth.random_constrained_state(N, 30 + net, B).astype(np.complex64).astype(np.complex128)
        o_ref, _ = M.forward(params, M.features(b))
        o = ctx.mlp_forward(net, B)
        rms = np.sqrt(np.mean(o_ref ** 2))
        assert np.max(np.abs(o - o_ref)) <= 2e-3 * rms
        L_ref, g_ref = M.loss_and_grads(params, b, a, N, K)
        L, g = ctx.mlp_loss_grad(net)
        assert L == pytest.approx(L_ref, rel=1e-4)
        gg = unflatten(g, N, H, K)
        for k in g_ref:
            x, y = gg[k].ravel(), g_ref[k].ravel()
            assert np.linalg.norm(x - y) <= 1e-2 * np.linalg.norm(y), k
            assert np.dot(x, y) / (np.linalg.norm(x) * np.linalg.norm(y)) >= 0.999, k


def test_learned_move_matches_oracle(oracle):
    N, S, T, reps, H, K = 8, 2, 3, 2, 32, 2
    temps = synth.geometric_temps(0.6, 1.4, T)
    ctx = mlp_ctx(N, S, T, reps, H, K, batch=8, temps=temps)
    ctx.init(5)
    ctx.mlp_setup([0, 2], seed=1)
    NP, Out = ctx.mlp_sizes()
    raw = [synth.random_mlp_params(2 * N, H, Out, seed=40 + n, out_scale=0.4) for n in range(2)]
    for n in range(2):
        ctx.mlp_set_params(n, raw[n])
    state = synth.random_constrained_state(N, 50, S * T * reps)
    ctx.set_state(state)
    ctx.resync()
    state32 = state.astype(np.complex64).astype(np.complex128)
    E, temp_of = ctx.energies()
    scale = 0.5
    ctx.mlp_move(scale)
    after = ctx.get_state().reshape(S * T * reps, N)
    ogs = [oracle.Graph(N, SEED3 + i) for i in range(S)]
    acc_seen = 0
    for n, t in enumerate([0, 2]):
        params = M.rounded(unflatten(raw[n], N, H, K))
        la, copies, prop = ctx.mlp_last_move(n)
        for b in range(S * reps):
            mu, r = divmod(b, reps)
            c = mu * T * reps + r * T + t  # copy holding temperature t (no swaps yet)
            assert copies[b] == c
            g, uc, ua = M.draws(5, 0, c, 2 * N - 1)  # run seed 5, first learned round
            a0 = state32[c][None]
            dH = lambda an: np.array([oracle.energy(ogs[mu], x) for x in an]) - oracle.energy(ogs[mu], state32[c])  # noqa
            an, la_ref, parts = M.move_log_alpha(params, a0, dH, 1.0 / temps[t], N, K, scale, g[None], np.array([uc]))
            np.testing.assert_allclose(prop[b], an[0], rtol=0, atol=2e-4)
            assert la[b] == pytest.approx(la_ref[0], abs=2e-3)
            accepted = math.log(ua) < la_ref[0]
            if abs(math.log(ua) - la_ref[0]) > 1e-2:  # decided away from the boundary
                np.testing.assert_allclose(after[c], an[0] if accepted else state32[c], rtol=0, atol=2e-4)
                acc_seen += int(accepted)
    a_cnt, tries = ctx.mlp_stats()
    assert np.all(tries == S * reps)


def test_learned_moves_keep_infinite_temperature_law():
    """Exact draws at beta ~ 0, then learned rounds only (no sweeps): the
    closed-form marginals of the reference law must stay put (this checks the
    GPU's reference-density and wrapped-density terms on their own)."""
    N, reps = 6, 512
    ctx = mlp_ctx(N, 1, 1, reps, 16, 2, batch=8, nets=1, temps=[1e7])
    ctx.init(9)
    ctx.mlp_setup([0], seed=4)
    for _ in range(40):
        ctx.mlp_move(0.5)
    acc, tries = ctx.mlp_stats()
    assert 0.1 < acc[0] / tries[0] < 0.98
    a = ctx.get_state().reshape(reps, N)
    ref = brute.beta0_moments(N)
    u = np.abs(a) ** 2
    assert np.mean(u) == pytest.approx(ref["E|a|^2"], abs=5 * u.std() / math.sqrt(u.size))
    assert np.mean(u ** 4) == pytest.approx(ref["E|a|^8"], abs=5 * (u ** 4).std() / math.sqrt(u.size))
    np.testing.assert_allclose(np.sum(np.abs(a) ** 4, axis=1), N, rtol=2e-5)


def test_harvest_train_and_learned_pt_are_unbiased(oracle):
    """Harvest pairs from PT, train, then run PT with learned rounds after every
    sweep: per-temperature <E>, C_V, <q^2> agree with the plain FP64 oracle
    within 2 sigma (jackknife over 8 samples) in >= 90% of cells, 4 sigma in all."""
    N, S, T, reps = 16, 8, 6, 2
    temps = synth.geometric_temps(0.5, 1.5, T)
    graphs = [rlpt.Graph(N, SEED3 + 50 + i) for i in range(S)]
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=2, mlp_hidden=64,
                   mlp_components=2, mlp_capacity=4096, mlp_batch=128, swap_interval=1, resync_interval=100,
                   measure_start=1000, measure_interval=1, n_bins=20)
    ctx.init(7)
    ctx.sweep(300)
    ctx.mlp_setup([1, 3], seed=2)
    ctx.mlp_harvest(rounds=200, lag=2)
    L0 = ctx.mlp_train(1, 1e-3)
    L1 = ctx.mlp_train(300, 1e-3)
    assert np.all(L1 < L0)
    ctx.mlp_enable(1, 0.5)
    ctx.sweep(4000 - ctx.counters()[0])
    ctx.check()
    acc, tries = ctx.mlp_stats()
    assert np.all(acc > 0)
    g = per_sample_obs(ctx.observables(), temps)
    ors = []
    for mu in range(S):
        pt = oracle.PT(oracle.Graph(N, SEED3 + 50 + mu), temps, n_reps=reps, run_seed=99, sample=mu,
                       swap_interval=1, resync_interval=100, measure_start=1000, measure_interval=1, n_bins=20)
        pt.run(4000)
        ors.append(pt)
    o = per_sample_obs(oracle_stack(ors), temps)
    cells = within2 = within4 = 0
    rep = []
    for k in ("E", "C_V", "q2", "Y2"):
        mg, sg = jackknife(g[k])
        mo, so = jackknife(o[k])
        z = np.abs(mg - mo) / np.sqrt(sg ** 2 + so ** 2)
        cells += z.size
        within2 += int(np.sum(z <= 2))
        within4 += int(np.sum(z <= 4))
        rep.append((k, np.round(z, 2)))
    assert within4 == cells, rep
    assert within2 >= 0.9 * cells, rep


def test_learned_rounds_replay_bitwise_in_hip_graphs():
    """Sweeps with learned rounds captured in HIP graph segments and replayed
    give bitwise the states, energies, observables and move counts of the same
    sweeps enqueued one by one (the learned kernels draw from a device move
    counter, so a replay advances the chain)."""
    N, S, T, reps = 16, 2, 4, 2
    temps = synth.geometric_temps(0.5, 1.5, T)
    graphs = [rlpt.Graph(N, SEED3 + 70 + i) for i in range(S)]
    ctxs = []
    for _ in range(2):
        ctx = make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=2, mlp_hidden=32,
                       mlp_components=2, mlp_capacity=256, mlp_batch=64, swap_interval=2, resync_interval=10,
                       measure_start=20, measure_interval=1, n_bins=16, series_len=64)
        ctx.init(3)
        ctx.sweep(20)
        ctx.mlp_setup([1, 2], seed=5)
        ctx.mlp_harvest(rounds=8, lag=1)
        ctx.mlp_train(20, 1e-3)
        ctx.mlp_enable(1, 0.3)
        ctx.sweep(30 - ctx.counters()[0] % 10)  # to a multiple of 10 sweeps
        ctxs.append(ctx)
    c1, c2 = ctxs
    c1.sweep(40)
    for _ in range(4):
        c2.run_graph(10, 1)
    assert np.array_equal(c1.get_state(), c2.get_state())
    assert np.array_equal(c1.energies()[0], c2.energies()[0])
    o1, o2 = c1.observables(), c2.observables()
    for f in o1:
        assert np.array_equal(o1[f], o2[f]), f
    a1, t1 = c1.mlp_stats()
    a2, t2 = c2.mlp_stats()
    assert np.array_equal(a1, a2) and np.array_equal(t1, t2) and np.all(t1 > 0)
    assert c1.counters() == c2.counters()


def test_training_lowers_held_out_nll_of_pt_displacements():
    """What training gains: on displacement pairs harvested from the PT run
    after training (never seen by it), the trained networks' negative
    log-likelihood is below that of the same networks at initialisation.  The
    τ_int-corrected comparison with plain PT is the benchmark's (it finds no
    speed-up); this checks that the networks do learn the harvested law."""
    N, S, T, reps = 16, 8, 6, 2
    temps = synth.geometric_temps(0.5, 1.5, T)
    graphs = [rlpt.Graph(N, SEED3 + 80 + i) for i in range(S)]
    Bm, Bt, rounds = S * reps, 128, 200
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=2, mlp_hidden=64,
                   mlp_components=2, mlp_capacity=rounds * Bm, mlp_batch=Bt, swap_interval=1, resync_interval=100)
    ctx.init(8)
    ctx.sweep(300)
    ctx.mlp_setup([1, 4], seed=6)
    ctx.mlp_harvest(rounds=rounds, lag=2)  # fills the store exactly: the next harvest starts at slot 0
    p0 = [ctx.mlp_get_params(n) for n in range(2)]
    ctx.mlp_train(400, 1e-3)
    p1 = [ctx.mlp_get_params(n) for n in range(2)]
    ctx.sweep(50)
    ctx.mlp_harvest(rounds=Bt // Bm, lag=2)  # fresh pairs in slots [0, Bt)
    for n in range(2):
        L1, _ = ctx.mlp_loss_grad(n)
        ctx.mlp_set_params(n, p0[n])
        L0, _ = ctx.mlp_loss_grad(n)
        ctx.mlp_set_params(n, p1[n])
        assert np.isfinite(L0) and np.isfinite(L1)
        assert L1 < L0 - 1.0, (n, L0, L1)


def _store_pairs(ctx, net, before, after):
    ctx.mlp_set_pairs(net, before, after)
    f32 = lambda v: v.astype(np.complex64).astype(np.complex128)  # noqa: E731
    return f32(before), f32(after)


def test_zero_amplitude_training_pairs_are_left_out():
    """Pairs with an exact zero amplitude (which the FP32 pair move can make)
    are left out of the training loss, as in the oracle: loss and gradients
    equal the oracle's over the other pairs, training stays finite, and a
    store with no usable pair is reported (RLPT_E_STATE), not trained on."""
    N, H, K, B = 8, 48, 3, 16
    ctx = mlp_ctx(N, 1, 2, 1, H, K, B, nets=1, cap=B)
    ctx.init(1)
    ctx.mlp_setup([0], seed=3)
    NP, Out = ctx.mlp_sizes()
    raw = synth.random_mlp_params(2 * N, H, Out, seed=12, out_scale=0.5)
    ctx.mlp_set_params(0, raw)
    before = synth.random_constrained_state(N, 22, B)
    after = synth.random_constrained_state(N, 32, B)
    before[3, 5] = 0.0
    after[7, N - 1] = 0.0
    after[9, 0] = 0.0
    b, a = _store_pairs(ctx, 0, before, after)
    params = M.rounded(unflatten(raw, N, H, K))
    L_ref, g_ref = M.loss_and_grads(params, b, a, N, K)
    L, g = ctx.mlp_loss_grad(0)
    assert np.isfinite(L) and L == pytest.approx(L_ref, rel=1e-4)
    gg = unflatten(g, N, H, K)
    for k in g_ref:
        x, y = gg[k].ravel(), g_ref[k].ravel()
        assert np.all(np.isfinite(x)), k
        assert np.linalg.norm(x - y) <= 1e-2 * np.linalg.norm(y), k
    L1 = ctx.mlp_train(20, 1e-3)
    assert np.all(np.isfinite(L1)) and np.all(np.isfinite(ctx.mlp_get_params(0)))
    dead = synth.random_constrained_state(N, 40, B)
    dead[:, 2] = 0.0
    ctx.mlp_set_pairs(0, dead, after)
    with pytest.raises(rlpt.RlptError) as e:
        ctx.mlp_train(1, 1e-3)
    assert e.value.code == rlpt.RLPT_E_STATE
    with pytest.raises(rlpt.RlptError):
        ctx.mlp_loss_grad(0)


def test_learned_move_from_a_zero_amplitude_is_rejected(oracle):
    """A learned item whose copy holds an exact zero amplitude is rejected
    (log acceptance -inf, state and energy untouched); the other items of the
    round follow the oracle as usual."""
    N, S, T, reps, H, K = 8, 2, 2, 2, 32, 2
    temps = synth.geometric_temps(0.6, 1.4, T)
    ctx = mlp_ctx(N, S, T, reps, H, K, batch=8, nets=1, temps=temps)
    ctx.init(5)
    ctx.mlp_setup([1], seed=1)
    state = synth.random_constrained_state(N, 51, S * T * reps)
    zero_copy = 0 * T * reps + 1 * T + 1  # sample 0, ladder 1, temperature 1
    state[zero_copy, 4] = 0.0
    ctx.set_state(state)
    ctx.resync()  # rescales the planted copy onto the constraint; its zero stays zero
    before = ctx.get_state().reshape(S * T * reps, N)
    assert before[zero_copy, 4] == 0.0
    E0, _ = ctx.energies()
    ctx.mlp_move(0.5)
    la, copies, _ = ctx.mlp_last_move(0)
    b = list(copies).index(zero_copy)
    assert la[b] == -np.inf
    assert np.all(np.isfinite(np.delete(la, b)))
    after = ctx.get_state().reshape(S * T * reps, N)
    assert np.array_equal(after[zero_copy], before[zero_copy])
    assert ctx.energies()[0][zero_copy] == E0[zero_copy]
    a_cnt, tries = ctx.mlp_stats()
    assert tries[0] == S * reps


def _infer_ctx(N, S, reps, H, K, batch, seed_graph=0):
    T = 2
    graphs = [rlpt.Graph(N, SEED3 + 200 + seed_graph + i) for i in range(S)]
    return mlp_ctx(N, S, T, reps, H, K, batch, nets=2, cap=max(batch, 64), graphs=graphs,
                   temps=synth.geometric_temps(0.7, 0.9, T))


@pytest.mark.parametrize("N,S,reps", [(64, 8, 2), (64, 12, 2), (256, 2, 8)])
def test_inference_forward_at_configured_size(N, S, reps):
    """The learned-proposal configurations' networks (2N -> 256 -> 256 ->
    4-component mixture: 1020 outputs at N = 64, 4092 at N = 256).  With
    samples x replicas = 16 the inference forward is the one-launch fused
    kernel (features formed in the kernel), otherwise the feature kernel and
    three GEMMs: outputs against the FP64 oracle on the same bfloat16
    operands, and bitwise against the training-path GEMMs on the same
    configurations; again after new parameters are set and after an Adam step
    (the fragment-order weight copy must follow both)."""
    H, K = 256, 4
    Bm = S * reps
    ctx = _infer_ctx(N, S, reps, H, K, batch=Bm)
    ctx.init(2)
    ctx.mlp_setup([0, 1], seed=7)
    NP, Out = ctx.mlp_sizes()
    assert Out == K * (4 * N - 1)
    states = synth.random_constrained_state(N, 60, Bm)
    b32, a32 = _store_pairs(ctx, 1, states, synth.random_constrained_state(N, 61, Bm))

    def check(net, raw):
        o = ctx.mlp_infer(net, states)
        params = M.rounded(unflatten(raw, N, H, K))
        o_ref, _ = M.forward(params, M.features(b32))
        rms = np.sqrt(np.mean(o_ref ** 2))
        assert np.max(np.abs(o - o_ref)) <= 2e-3 * rms
        return o

    raw = synth.random_mlp_params(2 * N, H, Out, seed=70, out_scale=0.5)
    ctx.mlp_set_params(1, raw)
    o = check(1, raw)
    assert np.array_equal(o, ctx.mlp_forward(1, Bm))  # the same bits as the three GEMMs
    raw2 = synth.random_mlp_params(2 * N, H, Out, seed=71, out_scale=0.5)
    ctx.mlp_set_params(1, raw2)
    check(1, raw2)
    ctx.mlp_set_pairs(0, states, synth.random_constrained_state(N, 62, Bm))
    ctx.mlp_train(1, 1e-2)  # one Adam step on both networks
    raw3 = ctx.mlp_get_params(1)
    assert not np.array_equal(raw3, raw2)
    o3 = check(1, raw3)
    assert np.array_equal(o3, ctx.mlp_forward(1, Bm))


@pytest.mark.parametrize("N", [64, 256])
def test_gradients_at_configured_size(N):
    """Training gradients of the configured networks (2N -> 256 -> 256 ->
    4-component mixture) on a minibatch of 512 pairs: every GEMM runs its
    multi-stage K loop (K = 128 or 512 inputs, 256 hidden, 512 rows for the
    weight gradients, 1020 or 4092 outputs for the input gradients).  Per
    tensor |g - g_ora| <= 1e-2 |g_ora| and cosine >= 0.999 against the FP64
    oracle on the same bfloat16 operands."""
    H, K, B = 256, 4, 512
    graphs = [rlpt.Graph(N, SEED3 + 300 + N)]
    ctx = mlp_ctx(N, 1, 2, 1, H, K, B, nets=1, cap=B, graphs=graphs)
    ctx.init(3)
    ctx.mlp_setup([0], seed=8)
    NP, Out = ctx.mlp_sizes()
    raw = synth.random_mlp_params(2 * N, H, Out, seed=80 + N, out_scale=0.5)
    ctx.mlp_set_params(0, raw)
    before = synth.random_constrained_state(N, 90 + N, B)
    after = synth.random_constrained_state(N, 91 + N, B)
    b, a = _store_pairs(ctx, 0, before, after)
    params = M.rounded(unflatten(raw, N, H, K))
    L_ref, g_ref = M.loss_and_grads(params, b, a, N, K)
    L, g = ctx.mlp_loss_grad(0)
    assert L == pytest.approx(L_ref, rel=1e-4)
    gg = unflatten(g, N, H, K)
    for k in g_ref:
        x, y = gg[k].ravel(), g_ref[k].ravel()
        assert np.linalg.norm(x - y) <= 1e-2 * np.linalg.norm(y), k
        assert np.dot(x, y) / (np.linalg.norm(x) * np.linalg.norm(y)) >= 0.999, k


@pytest.mark.parametrize("N,S,T,reps", [(64, 8, 4, 2), (256, 2, 4, 8)])
def test_learned_move_matches_oracle_at_configured_size(oracle, N, S, T, reps):
    """A learned round of the configured networks (H = 256, K = 4; samples x
    replicas = 16 items: the fused inference forward; at N = 256 the energy
    change runs over 128 term slices per sample) against the oracle on the
    same draws: proposals, log acceptance ratios and the decisions taken away
    from the boundary."""
    H, K = 256, 4
    temps = synth.geometric_temps(0.7, 1.0, T)
    graphs = [rlpt.Graph(N, SEED3 + 400 + i) for i in range(S)]
    ctx = mlp_ctx(N, S, T, reps, H, K, batch=16, nets=2, graphs=graphs, temps=temps)
    ctx.init(6)
    ctx.mlp_setup([1, 2], seed=2)
    NP, Out = ctx.mlp_sizes()
    raw = [synth.random_mlp_params(2 * N, H, Out, seed=140 + n, out_scale=0.05) for n in range(2)]
    for n in range(2):
        ctx.mlp_set_params(n, raw[n])
    state = synth.random_constrained_state(N, 150, S * T * reps)
    ctx.set_state(state)
    ctx.resync()
    state32 = state.astype(np.complex64).astype(np.complex128)
    scale = 0.05
    ctx.mlp_move(scale)
    after = ctx.get_state().reshape(S * T * reps, N)
    ogs = [oracle.Graph(N, SEED3 + 400 + i) for i in range(S)]
    decided = 0
    for n, t in enumerate([1, 2]):
        params = M.rounded(unflatten(raw[n], N, H, K))
        la, copies, prop = ctx.mlp_last_move(n)
        for b in range(S * reps):
            mu, r = divmod(b, reps)
            c = mu * T * reps + r * T + t
            assert copies[b] == c
            g, uc, ua = M.draws(6, 0, c, 2 * N - 1)
            E0 = oracle.energy(ogs[mu], state32[c])
            dH = lambda an: np.array([oracle.energy(ogs[mu], x) for x in an]) - E0  # noqa
            an, la_ref, parts = M.move_log_alpha(params, state32[c][None], dH, 1.0 / temps[t], N, K, scale, g[None],
                                                 np.array([uc]))
            np.testing.assert_allclose(prop[b], an[0], rtol=0, atol=5e-4)
            mag = abs(parts["lq_f"][0]) + abs(parts["lq_r"][0]) + abs(parts["dlogref"][0]) + abs(parts["dH"][0]) / temps[t]
            assert la[b] == pytest.approx(la_ref[0], abs=5e-3 + 2e-5 * mag), (n, b)
            if abs(math.log(ua) - la_ref[0]) > 2e-2 + 4e-5 * mag:
                accepted = math.log(ua) < la_ref[0]
                np.testing.assert_allclose(after[c], an[0] if accepted else state32[c], rtol=0, atol=5e-4)
                decided += 1
    assert decided >= S * reps  # most of the 32 decisions are away from the boundary


# ------------------------------------------------------------------ the subset move
def subset_ctx(N, S, T, reps, H, K, batch, m, nets=2, cap=64, graphs=None, temps=None, seed0=500):
    graphs = graphs or [rlpt.Graph(N, SEED3 + seed0 + i) for i in range(S)]
    temps = synth.geometric_temps(0.5, 1.5, T) if temps is None else temps
    return make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=nets, mlp_hidden=H,
                    mlp_components=K, mlp_capacity=cap, mlp_batch=batch, mlp_subset=m, resync_interval=0,
                    drift_tol=0.0), graphs


@pytest.mark.parametrize("N,S,T,reps,H,K,m,layout", [(16, 2, 3, 2, 32, 2, 4, rlpt.LAYOUT_CHUNKED),
                                                      (16, 2, 3, 2, 32, 2, 16, rlpt.LAYOUT_PACKED),
                                                      (64, 8, 4, 2, 256, 4, 8, rlpt.LAYOUT_AUTO)])
def test_subset_move_matches_oracle(oracle, N, S, T, reps, H, K, m, layout):
    """One subset round against the oracle on the same draws: the subset, the
    proposal (modes outside the subset untouched), the energy change summed
    from the subset's lists against the exact FP64 difference, the log
    acceptance ratio and the decisions away from the boundary."""
    temps = synth.geometric_temps(0.6, 1.2, T)
    graphs = [rlpt.Graph(N, SEED3 + 600 + i) for i in range(S)]
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=2, mlp_hidden=H,
                   mlp_components=K, mlp_capacity=64, mlp_batch=16, mlp_subset=m, resync_interval=0, drift_tol=0.0,
                   list_layout=layout)
    ctx.init(7)
    ctx.mlp_setup([1, 2], seed=3)
    NP, Out = ctx.mlp_sizes()
    raw = [synth.random_mlp_params(2 * N, H, Out, seed=160 + n, out_scale=0.3) for n in range(2)]
    for n in range(2):
        ctx.mlp_set_params(n, raw[n])
    state = synth.random_constrained_state(N, 170, S * T * reps)
    ctx.set_state(state)
    s32 = state.astype(np.complex64).astype(np.complex128)
    scale = 0.5
    ctx.mlp_move(scale)
    after = ctx.get_state().reshape(S * T * reps, N)
    ogs = [oracle.Graph(N, SEED3 + 600 + i) for i in range(S)]
    decided = 0
    for n, t in enumerate([1, 2]):
        params = M.rounded(unflatten(raw[n], N, H, K))
        la, copies, prop = ctx.mlp_last_move(n)
        for b in range(S * reps):
            mu, r = divmod(b, reps)
            c = mu * T * reps + r * T + t
            assert copies[b] == c
            Ss, g, uc, ua = M.subset_draws(7, 0, c, N, m)
            E0 = oracle.energy(ogs[mu], s32[c])
            dH = lambda an: oracle.energy(ogs[mu], an) - E0  # noqa
            an, la_ref, parts = M.subset_move_log_alpha(params, s32[c], Ss, dH, 1.0 / temps[t], N, K, scale, g, uc)
            rest = np.setdiff1d(np.arange(N), Ss)
            assert np.array_equal(prop[b][rest], s32[c][rest]), (n, b)
            np.testing.assert_allclose(prop[b], an, rtol=0, atol=5e-4)
            mag = abs(parts["lq_f"]) + abs(parts["lq_r"]) + abs(parts["dlogref"]) + abs(parts["dH"]) / temps[t]
            assert la[b] == pytest.approx(la_ref, abs=3e-3 + 2e-5 * mag), (n, b)
            if abs(math.log(ua) - la_ref) > 2e-2 + 4e-5 * mag:
                accepted = math.log(ua) < la_ref
                np.testing.assert_allclose(after[c], an if accepted else s32[c], rtol=0, atol=5e-4)
                decided += 1
    assert decided >= S * reps
    acc, tries = ctx.mlp_stats()
    assert np.all(tries == S * reps)


@pytest.mark.parametrize("m", [0, 64])
def test_learned_moves_at_the_largest_sizes(oracle, m):
    """The largest learned configuration the library accepts: N = 512 (a sparse
    graph of mean degree 16, packed lists), K = 8 components (the network's
    outputs, 16,376 floats, staged in LDS by the proposal and accept stages)
    and, for the subset move, the largest subset m = 64; one round against the
    oracle on the same draws."""
    N, S, T, reps, H, K, z = 512, 1, 3, 2, 128, 8, 16
    temps = synth.geometric_temps(0.6, 1.2, T)
    graphs = [rlpt.Graph(N, SEED3 + 700, mean_degree=z)]
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=2, mlp_hidden=H,
                   mlp_components=K, mlp_capacity=64, mlp_batch=16, mlp_subset=m, resync_interval=0, drift_tol=0.0)
    ctx.init(8)
    ctx.mlp_setup([1, 2], seed=4)
    NP, Out = ctx.mlp_sizes()
    assert Out == K * (2 * (2 * N - 1) + 1)
    raw = [synth.random_mlp_params(2 * N, H, Out, seed=190 + n, out_scale=0.05) for n in range(2)]
    for n in range(2):
        if m == 0:  # small output biases: over 1023 coordinates larger means would reject every move
            raw[n][-Out:] *= 0.02
        ctx.mlp_set_params(n, raw[n])
    state = synth.random_constrained_state(N, 191, S * T * reps)
    ctx.set_state(state)
    s32 = state.astype(np.complex64).astype(np.complex128)
    scale = 0.05 if m == 0 else 0.1
    ctx.mlp_move(scale)
    after = ctx.get_state().reshape(S * T * reps, N)
    og = oracle.Graph(N, SEED3 + 700, mean_degree=z)
    decided = 0
    for n, t in enumerate([1, 2]):
        params = M.rounded(unflatten(raw[n], N, H, K))
        la, copies, prop = ctx.mlp_last_move(n)
        for b in range(S * reps):
            c = b * T + t
            assert copies[b] == c
            E0 = oracle.energy(og, s32[c])
            if m == 0:
                g, uc, ua = M.draws(8, 0, c, 2 * N - 1)
                dH = lambda an: np.array([oracle.energy(og, x) for x in an]) - E0  # noqa
                an, la_ref, parts = M.move_log_alpha(params, s32[c][None], dH, 1.0 / temps[t], N, K, scale, g[None],
                                                     np.array([uc]))
                an, la_ref = an[0], la_ref[0]
                parts = {k: v[0] for k, v in parts.items()}
            else:
                Ss, g, uc, ua = M.subset_draws(8, 0, c, N, m)
                dH = lambda an: oracle.energy(og, an) - E0  # noqa
                an, la_ref, parts = M.subset_move_log_alpha(params, s32[c], Ss, dH, 1.0 / temps[t], N, K, scale, g,
                                                            uc)
                rest = np.setdiff1d(np.arange(N), Ss)
                assert np.array_equal(prop[b][rest], s32[c][rest]), (n, b)
            np.testing.assert_allclose(prop[b], an, rtol=0, atol=5e-4)
            mag = abs(parts["lq_f"]) + abs(parts["lq_r"]) + abs(parts["dlogref"]) + abs(parts["dH"]) / temps[t]
            assert la[b] == pytest.approx(la_ref, abs=5e-3 + 2e-5 * mag), (n, b)
            if abs(math.log(ua) - la_ref) > 2e-2 + 4e-5 * mag:
                accepted = math.log(ua) < la_ref
                np.testing.assert_allclose(after[c], an if accepted else s32[c], rtol=0, atol=5e-4)
                decided += 1
    assert decided >= 2
    acc, tries = ctx.mlp_stats()
    assert np.all(tries == S * reps)


@pytest.mark.parametrize("N,H,K,B,m", [(16, 48, 3, 16, 5), (64, 256, 4, 512, 8)])
def test_subset_gradients_match_oracle(N, H, K, B, m):
    """Training loss and gradients of the subset move (each minibatch item in
    the chart of its own subset, drawn from the training stream) against the
    FP64 oracle on the same bfloat16 operands."""
    ctx, _ = subset_ctx(N, 1, 2, 1, H, K, B, m, nets=1, cap=B)
    ctx.init(1)
    ctx.mlp_setup([0], seed=9)
    NP, Out = ctx.mlp_sizes()
    raw = synth.random_mlp_params(2 * N, H, Out, seed=180 + N, out_scale=0.5)
    ctx.mlp_set_params(0, raw)
    before = synth.random_constrained_state(N, 181 + N, B)
    after = synth.random_constrained_state(N, 182 + N, B)
    b, a = _store_pairs(ctx, 0, before, after)
    subsets = [M.train_subset(9, 0, 0, i, N, m) for i in range(B)]
    params = M.rounded(unflatten(raw, N, H, K))
    L_ref, g_ref = M.subset_loss_and_grads(params, b, a, subsets, N, K)
    L, g = ctx.mlp_loss_grad(0)
    assert L == pytest.approx(L_ref, rel=1e-4)
    gg = unflatten(g, N, H, K)
    for k in g_ref:
        x, y = gg[k].ravel(), g_ref[k].ravel()
        assert np.linalg.norm(x - y) <= 1e-2 * np.linalg.norm(y), k
        assert np.dot(x, y) / (np.linalg.norm(x) * np.linalg.norm(y)) >= 0.999, k


def test_subset_moves_keep_infinite_temperature_law():
    """Exact draws at beta ~ 0, then subset rounds only: the closed-form
    marginals of the reference law stay put."""
    N, reps = 6, 512
    ctx, _ = subset_ctx(N, 1, 1, reps, 16, 2, 8, 3, nets=1, temps=[1e7])
    ctx.init(9)
    ctx.mlp_setup([0], seed=4)
    for _ in range(40):
        ctx.mlp_move(0.8)
    acc, tries = ctx.mlp_stats()
    assert 0.1 < acc[0] / tries[0] < 0.98
    a = ctx.get_state().reshape(reps, N)
    ref = brute.beta0_moments(N)
    u = np.abs(a) ** 2
    assert np.mean(u) == pytest.approx(ref["E|a|^2"], abs=5 * u.std() / math.sqrt(u.size))
    assert np.mean(u ** 4) == pytest.approx(ref["E|a|^8"], abs=5 * (u ** 4).std() / math.sqrt(u.size))
    np.testing.assert_allclose(np.sum(np.abs(a) ** 4, axis=1), N, rtol=2e-5)


def test_subset_learned_pt_is_unbiased(oracle):
    """Harvest, train and run PT with a subset round after every sweep: the
    per-temperature laws agree with the plain FP64 oracle (the t-law rule)."""
    from tests.test_gpu_parity import check_same_law, same_law_report
    N, S, T, reps = 16, 8, 6, 2
    temps = synth.geometric_temps(0.5, 1.5, T)
    graphs = [rlpt.Graph(N, SEED3 + 650 + i) for i in range(S)]
    ctx = make_ctx(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, mlp_nets=2, mlp_hidden=64,
                   mlp_components=2, mlp_capacity=4096, mlp_batch=128, mlp_subset=4, swap_interval=1,
                   resync_interval=100, measure_start=1000, measure_interval=1, n_bins=20)
    ctx.init(7)
    ctx.sweep(300)
    ctx.mlp_setup([1, 3], seed=2)
    ctx.mlp_harvest(rounds=200, lag=2)
    L0 = ctx.mlp_train(1, 1e-3)
    L1 = ctx.mlp_train(300, 1e-3)
    assert np.all(L1 < L0)
    ctx.mlp_enable(1, 0.5)
    ctx.sweep(4000 - ctx.counters()[0])
    ctx.check()
    acc, tries = ctx.mlp_stats()
    assert np.all(acc > 0)
    g = per_sample_obs(ctx.observables(), temps)
    ors = []
    for mu in range(S):
        pt = oracle.PT(oracle.Graph(N, SEED3 + 650 + mu), temps, n_reps=reps, run_seed=98, sample=mu,
                       swap_interval=1, resync_interval=100, measure_start=1000, measure_interval=1, n_bins=20)
        pt.run(4000)
        ors.append(pt)
    o = per_sample_obs(oracle_stack(ors), temps)
    check_same_law(same_law_report(g, o, keys=("E", "C_V", "q2", "Y2")))
