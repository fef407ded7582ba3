"""CPU: the arithmetic behind the bench line's tau_int-corrected ratios and
its failed-network flags (bench.py), on constructed inputs."""
import numpy as np
import pytest

import bench


def test_ratio_of_equal_tau_is_the_rate_ratio():
    tau = np.array([[10.0, 20.0, 40.0], [5.0, 6.0, 7.0]])
    r = bench.eff_ratio(tau, tau, 300.0, 400.0)
    assert r["ratio"] == [0.75, 0.75]
    assert r["lo"] == r["hi"] == [0.75, 0.75]
    assert r["status"] == ["slower", "slower"]


def test_ratio_is_the_geometric_mean_of_per_sample_effective_rates():
    """eff = sweeps/s / (2 tau) per sample; the ratio is the geometric mean over
    samples of eff_a / eff_b, its band exp(+-1 standard error of the mean log)."""
    rng = np.random.default_rng(3)
    tau_b = rng.uniform(50, 500, size=(3, 8))
    tau_a = tau_b / rng.uniform(1.5, 4.0, size=(3, 8))
    sps_a, sps_b = 280.0, 384.0
    r = bench.eff_ratio(tau_a, tau_b, sps_a, sps_b)
    eff = (sps_a / (2 * tau_a)) / (sps_b / (2 * tau_b))
    lg = np.log(eff)
    ref = np.exp(lg.mean(axis=1))
    se = lg.std(axis=1, ddof=1) / np.sqrt(8)
    np.testing.assert_allclose(r["ratio"], ref, atol=1e-3)
    np.testing.assert_allclose(r["lo"], ref * np.exp(-se), atol=1e-3)
    np.testing.assert_allclose(r["hi"], ref * np.exp(se), atol=1e-3)
    for s, lo, hi in zip(r["status"], r["lo"], r["hi"]):
        assert s == ("faster" if lo > 1 else "slower" if hi < 1 else "unresolved")


def test_band_holding_one_is_unresolved():
    tau_b = np.array([[100.0, 100.0, 100.0, 100.0]])
    tau_a = np.array([[50.0, 200.0, 60.0, 180.0]])
    r = bench.eff_ratio(tau_a, tau_b, 1.0, 1.0)
    assert r["lo"][0] < 1 < r["hi"][0]
    assert r["status"] == ["unresolved"]


def test_dead_networks_flags_no_acceptance_and_nonfinite_losses():
    losses = np.array([[1.0, 2.0, np.nan], [0.5, 1.0, np.inf]])
    bad = bench.dead_networks([0.1, 0.0, 0.2], losses)
    assert bad == [{"network": 1, "failed": "accepted no learned move"},
                   {"network": 2, "failed": "non-finite training loss"}]
    assert bench.dead_networks([0.1, 0.2], None) == []


def test_paired_agreement_error_is_the_standard_error_of_the_paired_mean():
    """the jackknife error of a mean over samples equals its standard error"""
    rng = np.random.default_rng(5)
    b = rng.normal(size=(4, 8))
    a = b + rng.normal(0.3, 1.0, size=(4, 8))
    r = bench.paired_agreement(a, b)
    d = a - b
    np.testing.assert_allclose(r["diff"], d.mean(axis=1), atol=1e-4)
    np.testing.assert_allclose(r["err"], d.std(axis=1, ddof=1) / np.sqrt(8), atol=1e-4)
    z = np.abs(d.mean(axis=1)) / (d.std(axis=1, ddof=1) / np.sqrt(8))
    np.testing.assert_allclose(r["z"], z, atol=1e-2)
    assert r["within_2sigma"] == pytest.approx(np.mean(z <= 2))


def test_paired_agreement_sees_a_shift_that_the_sample_spread_hides():
    """pairing removes what the runs share: a small shift common to all samples
    stands out although the samples themselves differ far more"""
    rng = np.random.default_rng(6)
    b = rng.normal(0.0, 10.0, size=(3, 8))
    r0 = bench.paired_agreement(b + rng.normal(0.0, 0.01, size=(3, 8)), b)
    r1 = bench.paired_agreement(b + 0.1 + rng.normal(0.0, 0.01, size=(3, 8)), b)
    assert r0["within_2sigma"] == 1.0
    assert r1["within_2sigma"] == 0.0


def test_window_means_are_per_sample_means_over_the_window():
    rng = np.random.default_rng(7)
    o = {"series_e": rng.normal(size=(8, 6, 50)).astype(np.float32),
         "series_q": rng.uniform(-1, 1, size=(8, 6, 50)).astype(np.float32)}
    w = bench.window_means(o, [1, 4], 10, 40)
    assert w["E"].shape == w["q2"].shape == w["E_first"].shape == w["E_second"].shape == (2, 8)
    for i, t in enumerate([1, 4]):
        for mu in range(8):
            e = o["series_e"][mu, t].astype(np.float64)
            assert w["E"][i, mu] == pytest.approx(float(np.mean(e[10:40])))
            assert w["E_first"][i, mu] == pytest.approx(float(np.mean(e[10:25])))
            assert w["E_second"][i, mu] == pytest.approx(float(np.mean(e[25:40])))
            assert w["q2"][i, mu] == pytest.approx(float(np.mean(o["series_q"][mu, t, 10:40].astype(np.float64) ** 2)))
