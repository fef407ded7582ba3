"""Pins of the FP64 learned-proposal reference (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from tests import brute


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.uniform(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_single_gaussian_nll_closed_form():
    N, K = 3, 1
    D = 2 * N - 1
    rng = np.random.default_rng(1)
    o = rng.standard_normal((4, K * (2 * D + 1)))
    delta = rng.standard_normal((4, D))
    L, _ = M.nll_and_grad(o, delta, N, K)
    _, mu, sigma, _ = M.mixture(o, N, K)
    ref = np.mean(np.sum(np.log(sigma[:, 0]) + 0.5 * math.log(2 * math.pi)
                         + 0.5 * ((delta - mu[:, 0]) / sigma[:, 0]) ** 2, axis=1))
    assert L == pytest.approx(ref, rel=1e-12)


def test_nll_gradient_finite_differences():
    N, K = 3, 3
    rng = np.random.default_rng(2)
    _, D, Out = M.sizes(N, K)
    o = rng.standard_normal((5, Out))
    delta = rng.standard_normal((5, D)) * 0.5
    L, g = M.nll_and_grad(o, delta, N, K)
    h = 1e-6
    for idx in [(0, 0), (1, 2), (2, K + 3), (3, K + K * D + 4), (4, Out - 1)]:
        op, om = o.copy(), o.copy()
        op[idx] += h
        om[idx] -= h
        fd = (M.nll_and_grad(op, delta, N, K)[0] - M.nll_and_grad(om, delta, N, K)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_parameter_gradients_finite_differences(oracle):
    N, H, K = 4, 12, 2
    rng = np.random.default_rng(3)
    params = M.init_params(N, H, K, rng, out_scale=0.5)
    a = np.array([oracle.init_copy(N, 5, c) for c in range(6)])
    b = np.array([oracle.init_copy(N, 6, c) for c in range(6)])
    L, grads = M.loss_and_grads(params, a, b, N, K, gemm_bf16=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = params[name].reshape(-1)
        for i in rng.choice(flat.size, 4, replace=False):
            old = flat[i]
            flat[i] = old + h
            Lp, _ = M.loss_and_grads(params, a, b, N, K, gemm_bf16=False)
            flat[i] = old - h
            Lm, _ = M.loss_and_grads(params, a, b, N, K, gemm_bf16=False)
            flat[i] = old
            assert grads[name].reshape(-1)[i] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5, abs=1e-8), name


def test_bf16_operands_are_the_exact_network_on_rounded_inputs(oracle):
    """With bfloat16 matrix-product operands the forward equals the exact
    network evaluated layer by layer on rounded inputs (written out here with
    torch's bfloat16 conversion), and stays within bfloat16 resolution of the
    exact network; the backward's weight gradients are the exact gradient's
    products on rounded factors."""
    import torch
    N, H, K = 5, 24, 2
    rng = np.random.default_rng(8)
    params = M.rounded(M.init_params(N, H, K, rng, out_scale=0.5))
    a = np.array([oracle.init_copy(N, 9, c) for c in range(7)])
    X = M.features(a)

    def tb(v):
        return torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()

    h1 = M.silu(tb(X) @ params["W1"] + params["b1"])
    h2 = M.silu(tb(h1) @ params["W2"] + params["b2"])
    ref = tb(h2) @ params["W3"] + params["b3"]
    o, _ = M.forward(params, X)
    np.testing.assert_allclose(o, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    o_exact, _ = M.forward(params, X, gemm_bf16=False)
    assert np.max(np.abs(o - o_exact)) < 2e-2 * np.sqrt(np.mean(o_exact ** 2))
    assert np.max(np.abs(o - o_exact)) > 0.0
    b = np.array([oracle.init_copy(N, 10, c) for c in range(7)])
    _, g = M.loss_and_grads(params, a, b, N, K)
    _, g_exact = M.loss_and_grads(params, a, b, N, K, gemm_bf16=False)
    for k in g:
        assert np.linalg.norm(g[k] - g_exact[k]) <= 3e-2 * np.linalg.norm(g_exact[k]), k


def test_coordinates_roundtrip_and_constraint(oracle):
    a = np.array([oracle.init_copy(7, 3, c) for c in range(5)])
    y, psi, w = M.coords(a)
    b = M.from_coords(y, psi)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.sum(np.abs(b) ** 4, axis=1), 7.0, rtol=1e-13)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=1e-13)


def test_wrapped_proposal_density_integrates_to_one():
    """N = 2: one y coordinate and two phases; integrate q over R x T^2 on a grid."""
    N, K = 2, 2
    rng = np.random.default_rng(4)
    _, D, Out = M.sizes(N, K)
    o = rng.standard_normal((1, Out))
    o[0, K + K * D:] += 1.0  # wide phase components: the wrapping matters
    ys = np.linspace(-14, 14, 801)
    ps = np.linspace(-math.pi, math.pi, 97)[:-1]
    Y, P1, P2 = np.meshgrid(ys, ps, ps, indexing="ij")
    dy = Y.reshape(-1, 1)
    dpsi = np.stack([P1.reshape(-1), P2.reshape(-1)], axis=1)
    lq = M.log_q(np.repeat(o, dy.shape[0], axis=0), dy, dpsi, N, K, 1.0)
    total = np.exp(lq).sum() * (ys[1] - ys[0]) * (ps[1] - ps[0]) ** 2
    assert total == pytest.approx(1.0, rel=2e-3)


def _chain(oracle, N, beta, graph, n_chains, n_moves, scale, seed, H=16, K=2):
    """Learned moves only, from exact infinite-temperature draws.  Returns the
    history of states, of energies (None at beta = 0) and the acceptance rate."""
    rng = np.random.default_rng(seed)
    params = M.init_params(N, H, K, rng, out_scale=1.0)
    a = np.array([oracle.init_copy(N, seed, c) for c in range(n_chains)])
    _, D, _ = M.sizes(N, K)
    acc = 0
    hist, ehist = [], []
    q = None if graph is None else graph.quads.astype(np.int64)
    E = None if graph is None else brute.energy_batch(q, graph.J, a)
    for t in range(n_moves):
        g = rng.standard_normal((n_chains, D))
        uc = rng.uniform(size=n_chains)
        ua = rng.uniform(size=n_chains)
        dH = None if graph is None else (lambda an: brute.energy_batch(q, graph.J, an) - E)  # noqa: E731
        an, la, parts = M.move_log_alpha(params, a, dH, beta, N, K, scale, g, uc)
        ok = np.log(ua) < la
        a = np.where(ok[:, None], an, a)
        if graph is not None:
            E = np.where(ok, E + parts["dH"], E)
            ehist.append(E.copy())
        acc += ok.sum()
        hist.append(a.copy())
    return np.array(hist), (np.array(ehist) if ehist else None), acc / (n_chains * n_moves)


def test_learned_chain_keeps_infinite_temperature_law(oracle):
    """Starting from exact beta = 0 draws, learned moves alone must keep the
    closed-form marginals; a wrong reference-density (Jacobian) term would not."""
    N = 4
    hist, _, acc = _chain(oracle, N, 0.0, None, n_chains=3000, n_moves=30, scale=0.3, seed=7)
    assert 0.1 < acc < 0.95
    ref = brute.beta0_moments(N)
    u = np.abs(hist[10:]) ** 2
    per_t = u.mean(axis=(1, 2))
    assert per_t.mean() == pytest.approx(ref["E|a|^2"], abs=5 * u.std() / math.sqrt(3000 * N))
    u4 = (u ** 4).mean(axis=(1, 2))
    assert u4.mean() == pytest.approx(ref["E|a|^8"], abs=5 * (u ** 4).std() / math.sqrt(3000 * N))
    np.testing.assert_allclose(np.sum(np.abs(hist[-1]) ** 4, axis=1), N, rtol=1e-10)


@pytest.mark.slow
def test_learned_chain_samples_boltzmann_law(oracle):
    """At finite beta, learned moves alone (an untrained network) reproduce
    the importance-sampling reference <E> of the N = 4 comb (one term)."""
    N = 4
    g = oracle.Graph(N, 0, oracle.OMEGA_COMB)
    g.J = np.array([2.0])
    _, E, acc = _chain(oracle, N, 1.0, g, n_chains=1000, n_moves=900, scale=0.4, seed=8)
    ref, err = brute.importance_reference(g.quads.astype(np.int64), g.J, N, [1.0], M=1000000, seed=9)
    per_chain = E[400:].mean(axis=0)
    se = per_chain.std() / math.sqrt(len(per_chain))
    assert 0.2 < acc < 0.9
    assert per_chain.mean() == pytest.approx(ref["E"][0], abs=4 * math.sqrt(se ** 2 + err["E"][0] ** 2))


def test_training_pairs_outside_the_chart_are_left_out(oracle):
    """A training pair with an exact zero amplitude in either configuration has
    no displacement in the alr chart (log 0): the loss and its gradients are
    those of the remaining pairs alone, finite, and a minibatch with no pair
    inside the chart is an error."""
    N, H, K, B = 6, 16, 2, 8
    rng = np.random.default_rng(11)
    params = M.rounded(M.init_params(N, H, K, rng, out_scale=0.5))
    a = np.array([oracle.init_copy(N, 12, c) for c in range(B)])
    b = np.array([oracle.init_copy(N, 13, c) for c in range(B)])
    a[2, 3] = 0.0
    b[5, N - 1] = 0.0  # the alr reference mode
    b[6, 0] = 0.0      # the mode that fixes the gauge of the features
    with np.errstate(divide="ignore", invalid="ignore"):
        assert not np.all(np.isfinite(M.displacement(a, b)[[2, 5, 6]]))
    keep = np.array([i not in (2, 5, 6) for i in range(B)])
    L, g = M.loss_and_grads(params, a, b, N, K)
    L_ref, g_ref = M.loss_and_grads(params, a[keep], b[keep], N, K)
    assert np.isfinite(L) and L == L_ref
    for k in g:
        assert np.all(np.isfinite(g[k])) and np.array_equal(g[k], g_ref[k]), k
    with pytest.raises(ValueError):
        M.loss_and_grads(params, a[[2, 5]], b[[2, 5]], N, K)


def test_learned_moves_touching_the_chart_boundary_are_rejected(oracle):
    """A learned move from a configuration with a zero amplitude, or whose
    proposal underflows an intensity to zero, has log acceptance -inf; the
    other rows of the batch are unaffected (same ratio as alone)."""
    N, H, K = 5, 12, 2
    rng = np.random.default_rng(14)
    params = M.rounded(M.init_params(N, H, K, rng, out_scale=0.2))
    a = np.array([oracle.init_copy(N, 15, c) for c in range(4)])
    a[1, 2] = 0.0
    _, D, _ = M.sizes(N, K)
    g = rng.standard_normal((4, D))
    uc = rng.uniform(size=4)
    _, la, parts = M.move_log_alpha(params, a, None, 0.0, N, K, 0.5, g, uc)
    assert la[1] == -np.inf and not parts["inside"][1]
    assert np.all(np.isfinite(la[[0, 2, 3]]))
    _, la0, _ = M.move_log_alpha(params, a[[0]], None, 0.0, N, K, 0.5, g[[0]], uc[[0]])
    assert la0[0] == la[0]
    # a mean displacement of -3000 in y_0 (every component) underflows w'_0 to zero
    big = {k: v.copy() for k, v in params.items()}
    big["b3"][K + np.arange(K) * D] = -3000.0
    a2 = np.array([oracle.init_copy(N, 16, c) for c in range(2)])
    an, la2, parts2 = M.move_log_alpha(big, a2, None, 0.0, N, K, 1.0, g[:2], uc[:2])
    assert np.all(la2 == -np.inf) and not np.any(parts2["inside"])


# ------------------------------------------------------------------ the subset move
def test_subset_draw_is_a_uniform_subset():
    """The partial Fisher-Yates shuffle gives m distinct ascending modes, each
    mode with probability m/N and each pair of modes with m(m-1)/(N(N-1))
    (a uniform m-subset); m = N gives every mode."""
    N, m, n = 9, 3, 20000
    rng = np.random.default_rng(21)
    cnt = np.zeros(N)
    pair = np.zeros((N, N))
    for _ in range(n):
        S = M.subset_draw([int(x) for x in rng.integers(0, 2 ** 64, size=m, dtype=np.uint64)], N, m)
        assert len(set(S)) == m and np.all(np.diff(S) > 0)
        cnt[S] += 1
        pair[np.ix_(S, S)] += 1
    p = m / N
    assert np.all(np.abs(cnt / n - p) < 5 * math.sqrt(p * (1 - p) / n))
    q = m * (m - 1) / (N * (N - 1))
    off = pair[~np.eye(N, dtype=bool)] / n
    assert np.all(np.abs(off - q) < 5 * math.sqrt(q * (1 - q) / n))
    assert np.array_equal(M.subset_draw([5, 7, 9, 11, 13], 5, 5), np.arange(5))


def test_subset_move_changes_only_the_subset_and_keeps_the_constraint(oracle):
    N, H, K = 7, 12, 2
    rng = np.random.default_rng(22)
    params = M.rounded(M.init_params(N, H, K, rng, out_scale=0.5))
    a = oracle.init_copy(N, 23, 0)
    S = np.array([1, 4, 6])
    g = rng.standard_normal(5)
    an, la, parts = M.subset_move_log_alpha(params, a, S, None, 0.0, N, K, 0.7, g, 0.3)
    rest = np.setdiff1d(np.arange(N), S)
    assert np.array_equal(an[rest], a[rest])
    assert np.sum(np.abs(an) ** 4) == pytest.approx(N, rel=1e-12)
    assert np.sum(np.abs(an[S]) ** 4) == pytest.approx(np.sum(np.abs(a[S]) ** 4), rel=1e-12)
    du, dpsi = M.subset_displacement(a, an, S)
    np.testing.assert_allclose(du, parts["du"], atol=1e-12)
    np.testing.assert_allclose(M.wrap(dpsi - parts["dpsi"]), 0.0, atol=1e-12)
    assert np.isfinite(la)
    z = a.copy()
    z[4] = 0.0
    assert M.subset_move_log_alpha(params, z, S, None, 0.0, N, K, 0.7, g, 0.3)[1] == -np.inf
    assert np.isfinite(M.subset_move_log_alpha(params, z, np.array([0, 2, 3]), None, 0.0, N, K, 0.7, g, 0.3)[1])


def test_subset_proposal_density_integrates_to_one():
    """m = 2: one u coordinate and two phases; q over R x T^2 on a grid."""
    N, K = 5, 2
    rng = np.random.default_rng(24)
    _, D, Out = M.sizes(N, K)
    o = rng.standard_normal(Out)
    o[K + K * D:] += 1.0
    S = np.array([1, 3])
    us = np.linspace(-14, 14, 561)
    ps = np.linspace(-math.pi, math.pi, 73)[:-1]
    U, P1, P2 = np.meshgrid(us, ps, ps, indexing="ij")
    lq = M.subset_log_q(o, S, U.reshape(-1, 1), np.stack([P1.reshape(-1), P2.reshape(-1)], axis=1), N, K, 1.0)
    tot = np.exp(lq).sum() * (us[1] - us[0]) * (ps[1] - ps[0]) ** 2
    assert tot == pytest.approx(1.0, rel=3e-3)


def test_subset_nll_gradient_finite_differences(oracle):
    N, H, K = 5, 10, 2
    rng = np.random.default_rng(25)
    params = M.init_params(N, H, K, rng, out_scale=0.5)
    a = np.array([oracle.init_copy(N, 26, c) for c in range(6)])
    b = np.array([oracle.init_copy(N, 27, c) for c in range(6)])
    subsets = [np.sort(rng.choice(N, 3, replace=False)) for _ in range(6)]
    L, grads = M.subset_loss_and_grads(params, a, b, subsets, N, K, gemm_bf16=False)
    h = 1e-6
    for name in ("W1", "b2", "W3", "b3"):
        flat = params[name].reshape(-1)
        for i in rng.choice(flat.size, 4, replace=False):
            old = flat[i]
            flat[i] = old + h
            Lp, _ = M.subset_loss_and_grads(params, a, b, subsets, N, K, gemm_bf16=False)
            flat[i] = old - h
            Lm, _ = M.subset_loss_and_grads(params, a, b, subsets, N, K, gemm_bf16=False)
            flat[i] = old
            assert grads[name].reshape(-1)[i] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5, abs=1e-8), name


def _subset_chain(oracle, N, m, beta, graph, n_chains, n_moves, scale, seed, H=16, K=2):
    rng = np.random.default_rng(seed)
    params = M.init_params(N, H, K, rng, out_scale=1.0)
    a = np.array([oracle.init_copy(N, seed, c) for c in range(n_chains)])
    q = None if graph is None else graph.quads.astype(np.int64)
    E = None if graph is None else brute.energy_batch(q, graph.J, a)
    hist, ehist, acc = [], [], 0
    for _ in range(n_moves):
        for c in range(n_chains):
            S = np.sort(rng.choice(N, m, replace=False))
            g = rng.standard_normal(2 * m - 1)
            dH = None if graph is None else (lambda an: brute.energy_batch(q, graph.J, an[None])[0] - E[c])  # noqa
            an, la, parts = M.subset_move_log_alpha(params, a[c], S, dH, beta, N, K, scale, g, rng.uniform())
            if math.log(rng.uniform()) < la:
                a[c] = an
                acc += 1
                if graph is not None:
                    E[c] += parts["dH"]
        hist.append(a.copy())
        if graph is not None:
            ehist.append(E.copy())
    return np.array(hist), (np.array(ehist) if ehist else None), acc / (n_chains * n_moves)


def test_subset_chain_keeps_infinite_temperature_law(oracle):
    """Subset moves alone from exact beta = 0 draws keep the closed-form
    marginals: a wrong subset reference ratio or reverse density would not."""
    N, m = 5, 3
    hist, _, acc = _subset_chain(oracle, N, m, 0.0, None, n_chains=800, n_moves=25, scale=0.8, seed=28)
    assert 0.1 < acc < 0.95
    ref = brute.beta0_moments(N)
    u = np.abs(hist[5:]) ** 2
    assert u.mean() == pytest.approx(ref["E|a|^2"], abs=5 * u.std() / math.sqrt(800 * N))
    assert (u ** 4).mean() == pytest.approx(ref["E|a|^8"], abs=5 * (u ** 4).std() / math.sqrt(800 * N))


@pytest.mark.slow
def test_subset_chain_samples_boltzmann_law(oracle):
    """At finite beta, subset moves alone reproduce the importance-sampling
    reference <E> of the N = 4 comb (one term)."""
    N = 4
    g = oracle.Graph(N, 0, oracle.OMEGA_COMB)
    g.J = np.array([2.0])
    _, E, acc = _subset_chain(oracle, N, 2, 1.0, g, n_chains=200, n_moves=400, scale=0.8, seed=29)
    ref, err = brute.importance_reference(g.quads.astype(np.int64), g.J, N, [1.0], M=1000000, seed=30)
    per_chain = E[150:].mean(axis=0)
    se = per_chain.std() / math.sqrt(len(per_chain))
    assert 0.1 < acc < 0.95
    assert per_chain.mean() == pytest.approx(ref["E"][0], abs=4 * math.sqrt(se ** 2 + err["E"][0] ** 2))
