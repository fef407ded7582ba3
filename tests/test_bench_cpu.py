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
