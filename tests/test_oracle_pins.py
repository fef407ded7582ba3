"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check reaches the expected value by a route other than the oracle's own
code: numpy's Philox, itertools enumeration, a dense-tensor contraction,
finite differences, closed forms of the infinite-temperature law, and an
importance-sampling reference built from i.i.d. draws.
"""
import math

import numpy as np
import pytest
from scipy import stats

from tests import brute, synth


# --------------------------------------------------------------------------- generator
@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 7, 11, 13], [123456789, 987654321]),
    ([2 ** 64 - 1, 3, 2 ** 63, 9], [2 ** 64 - 1, 2 ** 64 - 1]),
    ([17, 0, 0, 0], [2511, 0x4752415048]),
])
def test_philox_matches_numpy(oracle, ctr, key):
    assert np.array_equal(oracle.philox(ctr, key), brute.numpy_philox_block(ctr, key))


# --------------------------------------------------------------------------- graph
@pytest.mark.parametrize("N,seed", [(6, 1), (9, 2), (12, 3), (16, 4), (16, 5)])
def test_graph_matches_enumeration(oracle, N, seed):
    g = oracle.Graph(N, seed)
    # frequencies: numpy's Philox words, top 53 bits, sorted (sec. II.C)
    ref_w = np.sort([(int(brute.numpy_philox_block([i, 0, 0, 0], [seed, 0x4752415048])[0]) >> 11) * 2.0 ** -53
                     for i in range(N)])
    assert np.array_equal(g.omega, ref_w)
    assert g.gamma == 1.0 / (2 * (N - 1))
    ref = brute.enumerate_terms(g.omega, g.gamma)
    assert np.array_equal(g.quads.astype(np.int64), ref)


def test_graph_split_mask(oracle):
    g = oracle.Graph(16, 7, split_mask=oracle.SPLIT_A)
    ref = brute.enumerate_terms(g.omega, g.gamma, split_mask=1)
    assert np.array_equal(g.quads.astype(np.int64), ref)


@pytest.mark.parametrize("N", list(range(4, 41)))
def test_comb_count_closed_form(oracle, N):
    g = oracle.Graph(N, 0, oracle.OMEGA_COMB)
    assert g.n_terms == brute.comb_count(N)
    # on the comb only the outer/inner split can match: i + l = j + k
    q = g.quads.astype(np.int64)
    assert np.all(q[:, 0] + q[:, 1] == q[:, 2] + q[:, 3])


def test_comb_n4_single_term(oracle):
    g = oracle.Graph(4, 0, oracle.OMEGA_COMB)
    assert g.n_terms == 1 and tuple(g.quads[0]) == (0, 3, 1, 2)


@pytest.mark.parametrize("N,seed", [(16, 11), (32, 12), (48, 13)])
def test_graph_structure(oracle, N, seed):
    g = oracle.Graph(N, seed)
    q = g.quads.astype(np.int64)
    # four distinct modes per term; conjugated pair and plain pair frequency-matched
    assert all(len(set(row)) == 4 for row in q)
    mism = (g.omega[q[:, 0]] + g.omega[q[:, 1]]) - (g.omega[q[:, 2]] + g.omega[q[:, 3]])
    assert np.all(np.abs(mism) < g.gamma)
    deg = np.bincount(q.ravel(), minlength=N)
    assert deg.sum() == 4 * g.n_terms
    # random frequencies keep about N(N-2)(N-3)/12 terms (keep prob ~ 4 gamma)
    expect = N * (N - 2) * (N - 3) / 12.0
    assert 0.6 * expect < g.n_terms < 1.4 * expect


def test_couplings_gaussian_with_variance_N_over_c(oracle):
    g = oracle.Graph(48, 21)
    sigma2 = 48.0 / g.n_terms
    z = g.J / math.sqrt(sigma2)
    n = len(z)
    assert abs(np.mean(z)) < 5.0 / math.sqrt(n)
    assert abs(np.var(z) - 1.0) < 6.0 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3


# --------------------------------------------------------------------------- energy
@pytest.mark.parametrize("N,seed", [(6, 1), (8, 2), (9, 3)])
def test_energy_matches_tensor_contraction(oracle, N, seed):
    g = oracle.Graph(N, seed)
    T = brute.coupling_tensor(N, g.quads, g.J)
    for s in range(3):
        a = synth.random_state(N, 100 + s)
        assert oracle.energy(g, a) == pytest.approx(brute.energy_tensor(T, a), rel=1e-12, abs=1e-12)


def test_energy_n4_comb_closed_form(oracle):
    g = oracle.Graph(4, 0, oracle.OMEGA_COMB)
    a = synth.random_state(4, 5)
    A, ph = np.abs(a), np.angle(a)
    ref = -2.0 * g.J[0] * np.prod(A) * math.cos(ph[1] + ph[2] - ph[0] - ph[3])
    assert oracle.energy(g, a) == pytest.approx(ref, rel=1e-13)


def test_energy_symmetries(oracle):
    g = oracle.Graph(16, 9)
    a = synth.random_state(16, 6)
    H = oracle.energy(g, a)
    assert oracle.energy(g, a * np.exp(0.7j)) == pytest.approx(H, rel=1e-12)
    assert oracle.energy(g, np.conj(a)) == pytest.approx(H, rel=1e-12)
    assert oracle.energy(g, 1.3 * a) == pytest.approx(1.3 ** 4 * H, rel=1e-12)
    # linear in the couplings
    g2 = oracle.Graph(16, 9)
    g2.J = 2.5 * g2.J
    assert oracle.energy(g2, a) == pytest.approx(2.5 * H, rel=1e-12)


# --------------------------------------------------------------------------- fields
@pytest.mark.parametrize("N,seed", [(8, 1), (16, 2)])
def test_fields_are_minus_half_gradient(oracle, N, seed):
    """dH/dRe a_l + i dH/dIm a_l = -2 F_l  (central differences)."""
    g = oracle.Graph(N, seed)
    a = synth.random_state(N, 7)
    F = oracle.fields(g, a)
    h = 1e-6
    for l in range(N):
        e = np.zeros(N, dtype=complex)
        e[l] = h
        dre = (oracle.energy(g, a + e) - oracle.energy(g, a - e)) / (2 * h)
        dim = (oracle.energy(g, a + 1j * e) - oracle.energy(g, a - 1j * e)) / (2 * h)
        assert complex(dre, dim) == pytest.approx(-2.0 * F[l], rel=1e-6, abs=1e-7)


def test_fields_energy_identity(oracle):
    """H = -1/2 sum_l Re(conj(a_l) F_l) for a degree-4 form."""
    g = oracle.Graph(24, 3)
    a = synth.random_state(24, 8)
    F = oracle.fields(g, a)
    assert -0.5 * np.sum(np.conj(a) * F).real == pytest.approx(oracle.energy(g, a), rel=1e-12)


# --------------------------------------------------------------------------- pair move
@pytest.mark.parametrize("N,seed", [(8, 1), (16, 2), (24, 3)])
def test_pair_dE_matches_brute_force(oracle, N, seed):
    g = oracle.Graph(N, seed)
    a = synth.random_state(N, 9)
    pairs = synth.random_pairs(N, 10, 40)
    new = synth.random_complex(11, 80)
    for t, (j, k) in enumerate(pairs):
        b = a.copy()
        b[j], b[k] = new[2 * t], new[2 * t + 1]
        ref = oracle.energy(g, b) - oracle.energy(g, a)
        got = oracle.pair_dE(g, a, int(j), int(k), new[2 * t], new[2 * t + 1])
        assert got == pytest.approx(ref, rel=1e-10, abs=1e-11)


@pytest.mark.parametrize("N,seed,m", [(12, 5, 4), (16, 6, 16), (24, 7, 9)])
def test_subset_energy_change_is_the_mode_by_mode_snapshot_sum(oracle, N, seed, m):
    """Changing the modes of a subset S (ascending) to new values changes H by
    sum_i -2 Re(conj(a'_i - a_i) F_i), F_i taken on the snapshot that holds
    the new values at the modes before s_i and the old ones elsewhere: exact,
    because every term holds a mode at most once (the identity the subset
    move's energy change is built on), checked against the brute-force
    difference of H."""
    g = oracle.Graph(N, seed)
    a = synth.random_state(N, 13 + seed)
    rng = np.random.default_rng(seed)
    S = np.sort(rng.choice(N, m, replace=False))
    new = synth.random_complex(14 + seed, m)
    b = a.copy()
    b[S] = new
    snap = a.copy()
    dE = 0.0
    for i, l in enumerate(S):
        F = oracle.fields(g, snap)
        dE += -2.0 * (np.conj(new[i] - a[l]) * F[l]).real
        snap[l] = new[i]
    assert dE == pytest.approx(oracle.energy(g, b) - oracle.energy(g, a), rel=1e-10, abs=1e-11)


def test_single_mode_reduction(oracle):
    """With a_k unchanged the pair formula is -2 Re(conj(delta_j) F_j)."""
    g = oracle.Graph(16, 4)
    a = synth.random_state(16, 12)
    F = oracle.fields(g, a)
    z = 0.3 - 0.8j
    got = oracle.pair_dE(g, a, 3, 9, z, a[9])
    assert got == pytest.approx(-2.0 * (np.conj(z - a[3]) * F[3]).real, rel=1e-12)


# --------------------------------------------------------------------------- beta = 0 law
def test_init_is_on_constraint_and_beta0_law(oracle):
    N = 12
    M = 20000
    a = np.array([oracle.init_copy(N, 77, c) for c in range(M)])
    s4 = np.sum(np.abs(a) ** 4, axis=1)
    assert np.max(np.abs(s4 - N)) < 1e-12 * N
    ref = brute.beta0_moments(N)
    u = np.abs(a) ** 2
    assert np.mean(u) == pytest.approx(ref["E|a|^2"], abs=4 * np.std(u) / math.sqrt(u.size))
    assert np.mean(u ** 4) == pytest.approx(ref["E|a|^8"], abs=4 * np.std(u ** 4) / math.sqrt(u.size) * 3)
    # phases uniform: mean of exp(i phi) ~ 0
    assert abs(np.mean(a / np.abs(a))) < 5.0 / math.sqrt(a.size)


def test_spectrum_is_flat_at_infinite_temperature(oracle):
    """The intensity spectrum accumulator I(omega_k) = <|a_k|^2> (sec. II.C):
    at infinite temperature every mode has the closed-form mean E|a|^2 of the
    flat constrained law, whatever its frequency, and at a finite temperature
    its sum over modes per measurement stays between the bounds of the
    constraint: 1 <= sum |a|^2 <= N (Cauchy-Schwarz with sum |a|^4 = N) times
    the measurement count."""
    N, reps = 6, 48
    g = oracle.Graph(N, 11)
    pt = oracle.PT(g, [1e11, 1e12], n_reps=reps, run_seed=5, swap_interval=1, resync_interval=0,
                   measure_start=0, measure_interval=1)
    pt.run(3000)
    ref = brute.beta0_moments(N)["E|a|^2"]
    spec = pt.acc["spectrum"] / pt.acc["e_n"][:, None]
    assert spec.shape == (2, N)
    # copies are independent: the error of a mode's mean from the per-copy spread over a long run
    tol = 5 * np.sqrt((ref * ref * 0.6) / (reps * 3000 / 3.0))
    np.testing.assert_allclose(spec, ref, rtol=0, atol=tol)
    cold = oracle.PT(g, [0.3, 0.6], n_reps=2, run_seed=6, swap_interval=1, resync_interval=0, measure_start=0,
                     measure_interval=1)
    cold.run(300)
    tot = cold.acc["spectrum"].sum(axis=1)
    assert np.all(tot >= cold.acc["e_n"] * 1.0 - 1e-9) and np.all(tot <= cold.acc["e_n"] * N + 1e-9)


def test_intensity_histogram_at_infinite_temperature(oracle):
    """P(I), the histogram of I / N on [0, 1] (sec. II.B): at infinite
    temperature its mean and second moment (bin centres, 400 bins) are the
    closed forms of the flat constrained law, E I/N = E|a|^2 and
    E (I/N)^2 = (N + 2N(N-1)/pi)/N^2; no mass lies outside [1/sqrt(N), 1]
    (sum|a|^2 >= sqrt(sum|a|^4) and Cauchy-Schwarz).  Binning I instead of
    I / N, or the overlap's bin rule, would fail all three."""
    N, reps, B, sweeps = 8, 64, 400, 2000
    g = oracle.Graph(N, 12)
    pt = oracle.PT(g, [1e11, 1e12], n_reps=reps, run_seed=4, swap_interval=1, resync_interval=0,
                   measure_start=0, measure_interval=1, n_bins=B)
    pt.run(sweeps)
    ref = brute.beta0_moments(N)
    h = pt.acc["hist_I"]
    assert np.all(h.sum(axis=1) == pt.acc["e_n"])
    centre = (np.arange(B) + 0.5) / B
    lo = int(math.floor(B / math.sqrt(N)))
    assert np.all(h[:, :lo] == 0)
    var = ref["E (I/N)^2"] - ref["E I/N"] ** 2
    n_eff = reps * sweeps / 3.0  # the per-copy series decorrelates within a few sweeps at beta = 0
    for t in range(2):
        p = h[t] / h[t].sum()
        m1 = float(np.sum(p * centre))
        m2 = float(np.sum(p * centre ** 2))
        assert m1 == pytest.approx(ref["E I/N"], abs=5 * math.sqrt(var / n_eff) + 1e-5)
        assert m2 == pytest.approx(ref["E (I/N)^2"], abs=10 * math.sqrt(var / n_eff) + 1.0 / (12 * B * B))
    cold = oracle.PT(g, [0.3, 0.6], n_reps=2, run_seed=6, swap_interval=1, resync_interval=0, measure_start=0,
                     measure_interval=1, n_bins=B)
    cold.run(500)
    assert np.all(cold.acc["hist_I"][:, :lo] == 0)


def test_beta0_chain_preserves_law_and_constraint(oracle):
    """At infinite temperature every move is accepted; starting from the exact
    beta = 0 law the chain must stay on it (the two-mode proposal is exactly
    uniform with respect to the constrained flat measure)."""
    N = 8
    g = oracle.Graph(N, 5)
    pt = oracle.PT(g, [1e12], n_reps=64, run_seed=3, swap_interval=1, resync_interval=0,
                   measure_start=0, measure_interval=1)
    ref = brute.beta0_moments(N)
    us, qs = [], []
    for _ in range(400):
        pt.run(5)
        u = np.abs(pt.a) ** 2
        us.append(u.copy())
        qs.append(np.sum(np.conj(pt.a[0::2]) * pt.a[1::2], axis=1).real / N)
    us = np.array(us)
    s4 = np.sum(us ** 2, axis=2)
    assert np.max(np.abs(s4 - N)) < 1e-10
    assert np.all(pt.acc["acc"] == pt.acc["tries"])
    # block errors over the 64 independent copies
    per_copy = us.mean(axis=(0, 2))
    assert np.mean(per_copy) == pytest.approx(ref["E|a|^2"], abs=5 * per_copy.std() / 8)
    per_copy8 = (us ** 4).mean(axis=(0, 2))
    assert np.mean(per_copy8) == pytest.approx(ref["E|a|^8"], abs=5 * per_copy8.std() / 8)
    q2 = (np.array(qs) ** 2).mean(axis=0)
    assert np.mean(q2) == pytest.approx(ref["Var q"], abs=5 * q2.std() / math.sqrt(len(q2)))


def test_high_temperature_expansion(oracle):
    """<H>_beta = -beta Var0(H) + O(beta^2) at small beta."""
    N = 10
    g = oracle.Graph(N, 8)
    v0 = brute.var0_energy(N, g.J)
    T = 20.0
    pt = oracle.PT(g, [T], n_reps=32, run_seed=4, swap_interval=1000000, resync_interval=0,
                   measure_start=200, measure_interval=2)
    pt.run(4200)
    mean = pt.acc["e_sum"][0] / pt.acc["e_n"][0]
    var = pt.acc["e_sq"][0] / pt.acc["e_n"][0] - mean ** 2
    assert var == pytest.approx(v0, rel=0.05)
    err = math.sqrt(v0 / pt.acc["e_n"][0]) * 3.0  # generous: correlated samples
    assert mean == pytest.approx(-v0 / T, abs=4 * err + 0.05 * v0 / T)


# --------------------------------------------------------------------------- parallel tempering
def _pt_stats(oracle, g, temps, seeds, n_sweeps, burn):
    rows = []
    for s in seeds:
        pt = oracle.PT(g, temps, n_reps=2, run_seed=s, swap_interval=1, resync_interval=100,
                       measure_start=burn, measure_interval=1, n_bins=40)
        pt.run(n_sweeps)
        A = pt.acc
        rows.append(dict(E=A["e_sum"] / A["e_n"], E2=A["e_sq"] / A["e_n"], y2=A["y2_sum"] / A["e_n"],
                         y4=A["y4_sum"] / A["e_n"], q2=A["q_sq"] / A["q_n"], q4=A["q_4"] / A["q_n"],
                         hist=A["hist"], hist_I=A["hist_I"], swap=A["swap_acc"] / A["swap_tries"]))
    return rows


@pytest.mark.slow
def test_pt_matches_importance_sampling(oracle):
    """Per-temperature energy, specific heat, IPR and overlap moments of the
    PT oracle agree with an importance-sampling reference built from i.i.d.
    infinite-temperature draws (independent of the Markov chain)."""
    N = 8
    g = oracle.Graph(N, 31)
    temps = np.array([1.0, 1.25, 1.55, 1.95, 2.4])
    ref, ref_err = brute.importance_reference(g.quads.astype(np.int64), g.J, N, temps, M=1000000, seed=5,
                                              i_bins=40)
    rows = _pt_stats(oracle, g, temps, seeds=range(1, 9), n_sweeps=12000, burn=1000)
    for key in ("E", "y2", "y4", "q2"):
        vals = np.array([r[key] for r in rows])
        m, se = vals.mean(axis=0), vals.std(axis=0, ddof=1) / math.sqrt(len(rows))
        tol = 4.5 * np.sqrt(se ** 2 + ref_err[key] ** 2)
        assert np.all(np.abs(m - ref[key]) < tol), (key, m, ref[key], se, ref_err[key])
    cv = np.array([(r["E2"] - r["E"] ** 2) / temps ** 2 for r in rows])
    cv_ref = (ref["E2"] - ref["E"] ** 2) / temps ** 2
    cv_err = np.sqrt(ref_err["E2"] ** 2 + (2 * ref["E"] * ref_err["E"]) ** 2) / temps ** 2
    m, se = cv.mean(axis=0), cv.std(axis=0, ddof=1) / math.sqrt(len(rows))
    assert np.all(np.abs(m - cv_ref) < 4.5 * np.sqrt(se ** 2 + cv_err ** 2)), (m, cv_ref, se, cv_err)
    # P(I): every bin's probability against the reweighted i.i.d. draws
    pI = np.array([r["hist_I"] / r["hist_I"].sum(axis=1, keepdims=True) for r in rows])
    m, se = pI.mean(axis=0), pI.std(axis=0, ddof=1) / math.sqrt(len(rows))
    tol = 4.5 * np.sqrt(se ** 2 + ref_err["pI"] ** 2) + 2e-4
    assert np.all(np.abs(m - ref["pI"]) < tol), (np.max(np.abs(m - ref["pI"]) / tol))


def test_overlap_histogram_is_symmetric_and_complete(oracle):
    """P_J(q) is symmetric (global phase a -> -a maps q -> -q) and holds one
    count per measurement and replica pair."""
    N = 12
    g = oracle.Graph(N, 2)
    temps = synth.geometric_temps(1.5, 3.0, 4)
    pt = oracle.PT(g, temps, n_reps=2, run_seed=9, measure_start=200, measure_interval=1, n_bins=10)
    pt.run(10200)
    h = pt.acc["hist"]
    assert np.all(h.sum(axis=1) == pt.n_meas)
    for t in range(4):
        p = h[t] / h[t].sum()
        asym = np.abs(p - p[::-1]).sum()
        assert asym < 0.12, (t, asym)


def test_swap_equal_temperatures_always_accepted(oracle):
    g = oracle.Graph(8, 3)
    pt = oracle.PT(g, [1.0, 1.0 + 1e-13, 1.0 + 2e-13], n_reps=2, run_seed=1, swap_interval=1)
    pt.run(200)
    assert np.all(pt.acc["swap_acc"] == pt.acc["swap_tries"])
    assert pt.acc["swap_tries"][0] == 200 * 2


def test_running_energy_has_no_drift(oracle):
    g = oracle.Graph(16, 6)
    pt = oracle.PT(g, synth.geometric_temps(0.3, 1.5, 4), n_reps=2, run_seed=2, resync_interval=250)
    drift = pt.run(1000)
    assert drift < 1e-11
    for c in range(pt.R):
        assert pt.E[c] == pytest.approx(oracle.energy(g, pt.a[c]), rel=1e-11, abs=1e-11)
        assert np.sum(np.abs(pt.a[c]) ** 4) == pytest.approx(16.0, rel=1e-12)


def test_ipr_bounds_and_identity(oracle):
    """Y_2 = N / I^2 on the constraint surface; 1/N <= Y_n <= 1."""
    g = oracle.Graph(12, 4)
    pt = oracle.PT(g, [0.5, 1.0], n_reps=2, run_seed=3, measure_start=0)
    pt.run(300)
    y2 = pt.acc["y2_sum"] / pt.acc["e_n"]
    y4 = pt.acc["y4_sum"] / pt.acc["e_n"]
    assert np.all((y2 >= 1 / 12) & (y2 <= 1)) and np.all((y4 >= 1 / 12) & (y4 <= 1))
    for c in range(pt.R):
        I = np.sum(np.abs(pt.a[c]) ** 2)
        S2 = np.sum(np.abs(pt.a[c]) ** 4)
        assert S2 / I ** 2 == pytest.approx(12 / I ** 2, rel=1e-12)


def test_shared_pair_schedule_same_law(oracle):
    """Sharing one pair sequence between the copies of a sample leaves each
    chain's transition kernel unchanged; energies agree with the default."""
    N = 8
    g = oracle.Graph(N, 31)
    temps = np.array([1.0, 1.5])
    res = []
    for shared in (False, True):
        Es = []
        for s in range(6):
            pt = oracle.PT(g, temps, n_reps=2, run_seed=100 + s, shared_pairs=shared, measure_start=500)
            pt.run(6000)
            Es.append(pt.acc["e_sum"] / pt.acc["e_n"])
        res.append(np.array(Es))
    d = res[0].mean(0) - res[1].mean(0)
    se = np.sqrt(res[0].var(0, ddof=1) / 6 + res[1].var(0, ddof=1) / 6)
    assert np.all(np.abs(d) < 4 * se + 0.02)


def test_pt_is_deterministic_and_thread_independent(oracle):
    g = oracle.Graph(16, 8)
    temps = synth.geometric_temps(0.3, 1.5, 6)
    out = []
    for nt in (1, 4):
        pt = oracle.PT(g, temps, n_reps=2, run_seed=5, n_threads=nt)
        pt.run(50)
        out.append((pt.a.copy(), pt.E.copy(), pt.temp_of.copy()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


# --------------------------------------------------------------------------- spherical constraint (rho = 2)
def test_rho2_init_on_sphere_and_beta0_law(oracle):
    """rho = 2 (sum |a|^2 = N, the spherical constraint the paper compares
    with): the initial draw is the uniform law on the complex sphere."""
    N = 12
    M = 20000
    a = np.array([oracle.init_copy(N, 78, c, rho=2) for c in range(M)])
    s2 = np.sum(np.abs(a) ** 2, axis=1)
    assert np.max(np.abs(s2 - N)) < 1e-12 * N
    ref = brute.beta0_moments_sphere(N)
    u = np.abs(a) ** 2
    assert np.mean(u ** 2) == pytest.approx(ref["E|a|^4"], abs=4 * np.std(u ** 2) / math.sqrt(u.size))
    assert np.mean(u ** 4) == pytest.approx(ref["E|a|^8"], abs=4 * np.std(u ** 4) / math.sqrt(u.size) * 3)
    assert abs(np.mean(a / np.abs(a))) < 5.0 / math.sqrt(a.size)


def test_rho2_beta0_chain_preserves_law_and_constraint(oracle):
    """rho = 2 at infinite temperature: the chain keeps sum |a|^2 = N and the
    uniform law on the sphere (intensity moments, overlap variance 1/(2N)).
    Drawing theta uniform with A' = (K cos theta, K sin theta) instead would
    put the pair's intensity split on the arcsine law, E|a|^4 -> 3N / (N+2)
    instead of 2N / (N+1): this pin tells the two apart."""
    N = 8
    g = oracle.Graph(N, 5)
    pt = oracle.PT(g, [1e12], n_reps=64, run_seed=3, swap_interval=1, resync_interval=0,
                   measure_start=0, measure_interval=1, rho=2)
    ref = brute.beta0_moments_sphere(N)
    us, qs = [], []
    for _ in range(400):
        pt.run(5)
        u = np.abs(pt.a) ** 2
        us.append(u.copy())
        qs.append(np.sum(np.conj(pt.a[0::2]) * pt.a[1::2], axis=1).real / N)
    us = np.array(us)
    assert np.max(np.abs(np.sum(us, axis=2) - N)) < 1e-10
    assert np.all(pt.acc["acc"] == pt.acc["tries"])
    per_copy4 = (us ** 2).mean(axis=(0, 2))
    assert np.mean(per_copy4) == pytest.approx(ref["E|a|^4"], abs=5 * per_copy4.std() / 8)
    assert abs(np.mean(per_copy4) - 3.0 * N / (N + 2.0)) > 5 * per_copy4.std() / 8
    per_copy8 = (us ** 4).mean(axis=(0, 2))
    assert np.mean(per_copy8) == pytest.approx(ref["E|a|^8"], abs=5 * per_copy8.std() / 8)
    q2 = (np.array(qs) ** 2).mean(axis=0)
    assert np.mean(q2) == pytest.approx(ref["Var q"], abs=5 * q2.std() / math.sqrt(len(q2)))


def test_rho2_high_temperature_expansion(oracle):
    """rho = 2: <H>_beta = -beta Var0(H) + O(beta^2), Var0 on the sphere."""
    N = 10
    g = oracle.Graph(N, 8)
    v0 = brute.var0_energy_sphere(N, g.J)
    T = 20.0
    pt = oracle.PT(g, [T], n_reps=32, run_seed=4, swap_interval=1000000, resync_interval=0,
                   measure_start=200, measure_interval=2, rho=2)
    pt.run(4200)
    mean = pt.acc["e_sum"][0] / pt.acc["e_n"][0]
    var = pt.acc["e_sq"][0] / pt.acc["e_n"][0] - mean ** 2
    assert var == pytest.approx(v0, rel=0.05)
    err = math.sqrt(v0 / pt.acc["e_n"][0]) * 3.0
    assert mean == pytest.approx(-v0 / T, abs=4 * err + 0.05 * v0 / T)


def test_rho2_resync_restores_sphere(oracle):
    """A state off the sphere by 3% keeps its norm through the moves (each
    preserves |a_j|^2 + |a_k|^2) and is rescaled onto sum |a|^2 = N at the
    recomputation, with the running energy reset to H of the rescaled state."""
    N = 9
    g = oracle.Graph(N, 6)
    pt = oracle.PT(g, [0.7], n_reps=1, run_seed=2, resync_interval=1, renorm_tol=1e-9, rho=2)
    pt.a[:] *= 1.015
    pt.E[0] = oracle.energy(g, pt.a[0])
    pt.run(1)
    assert np.sum(np.abs(pt.a[0]) ** 2) == pytest.approx(N, rel=1e-12)
    assert pt.E[0] == pytest.approx(oracle.energy(g, pt.a[0]), rel=1e-10, abs=1e-12)


@pytest.mark.slow
def test_rho2_pt_matches_importance_sampling(oracle):
    """rho = 2 PT against importance sampling from uniform draws on the sphere."""
    N = 8
    g = oracle.Graph(N, 31)
    temps = np.array([1.0, 1.4, 2.0])
    ref, ref_err = brute.importance_reference(g.quads.astype(np.int64), g.J, N, temps, M=600000, seed=6,
                                              draw=brute.beta0_draw_sphere)
    rows = []
    for s in range(1, 7):
        pt = oracle.PT(g, temps, n_reps=2, run_seed=s, swap_interval=1, resync_interval=100,
                       measure_start=1000, measure_interval=1, n_bins=40, rho=2)
        pt.run(10000)
        A = pt.acc
        rows.append(dict(E=A["e_sum"] / A["e_n"], y2=A["y2_sum"] / A["e_n"], q2=A["q_sq"] / A["q_n"]))
    for key in ("E", "y2", "q2"):
        vals = np.array([r[key] for r in rows])
        m, se = vals.mean(axis=0), vals.std(axis=0, ddof=1) / math.sqrt(len(rows))
        tol = 4.5 * np.sqrt(se ** 2 + ref_err[key] ** 2)
        assert np.all(np.abs(m - ref[key]) < tol), (key, m, ref[key], se, ref_err[key])


# --------------------------------------------------------------------------- sparse mode-locked graphs
@pytest.mark.parametrize("N,z,seed", [(16, 8, 1), (64, 8, 2), (200, 12, 3)])
def test_sparse_graph_terms(oracle, N, z, seed):
    """floor(z N / 4) terms, each with four distinct modes, frequency matched
    and kept once; mean degree z."""
    g = oracle.Graph(N, seed, mean_degree=z)
    assert g.n_terms == z * N // 4
    q = g.quads.astype(np.int64)
    assert np.all(np.sort(q, axis=1)[:, 1:] != np.sort(q, axis=1)[:, :-1])
    w = g.omega
    assert np.all(np.abs(w[q[:, 0]] + w[q[:, 1]] - w[q[:, 2]] - w[q[:, 3]]) < g.gamma)
    assert len({tuple(t) for t in q.tolist()}) == g.n_terms
    deg = np.bincount(q.ravel(), minlength=N)
    assert deg.sum() == 4 * g.n_terms


def test_sparse_graph_is_uniform_subset_of_complete_graph(oracle):
    """Every sparse term is a term of the complete mode-locked graph of the
    same frequencies, and the kept terms are a uniform sample of it: their
    normalised ranks in the complete graph's term order are uniform on [0, 1)
    (Kolmogorov-Smirnov over 300 disorder samples)."""
    from scipy import stats
    N, z = 14, 8
    ranks = []
    for seed in range(300):
        dense = oracle.Graph(N, seed)
        sparse = oracle.Graph(N, seed, mean_degree=z)
        index = {tuple(t): i for i, t in enumerate(dense.quads.tolist())}
        assert sparse.n_terms <= dense.n_terms
        for t in sparse.quads.tolist():
            assert tuple(t) in index
            ranks.append((index[tuple(t)] + 0.5) / dense.n_terms)
    assert stats.kstest(ranks, "uniform").pvalue > 1e-3


def test_sparse_graph_high_temperature_expansion(oracle):
    """PT on a sparse graph obeys the same high-temperature law as on the
    complete graph: Var0(H) = 8N / (pi^2 (N+2)) sum J^2 depends only on the
    term set being distinct quadruplets."""
    N = 48
    g = oracle.Graph(N, 9, mean_degree=6)
    v0 = brute.var0_energy(N, g.J)
    T = 20.0
    pt = oracle.PT(g, [T], n_reps=32, run_seed=4, swap_interval=1000000, resync_interval=0,
                   measure_start=200, measure_interval=2)
    pt.run(3200)
    mean = pt.acc["e_sum"][0] / pt.acc["e_n"][0]
    var = pt.acc["e_sq"][0] / pt.acc["e_n"][0] - mean ** 2
    assert var == pytest.approx(v0, rel=0.05)
    err = math.sqrt(v0 / pt.acc["e_n"][0]) * 3.0
    assert mean == pytest.approx(-v0 / T, abs=4 * err + 0.05 * v0 / T)
