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


def _csv(path, header, rows):
    import csv
    import os
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_fabric_traffic_is_the_counters_scaled_by_the_copy_calibration(tmp_path, monkeypatch):
    """The roofline's traffic: FETCH_SIZE and WRITE_SIZE of the sweep kernel (KiB
    per dispatch), each scaled by the bytes a 512 MiB device copy moves over
    what the same counter reads for it; constructed rocprofv3 CSVs."""
    import json
    import os
    root = tmp_path / "repo"
    d = root / "gpurun_out" / "prof"
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(root / "profiles" / "traffic.json"))
    monkeypatch.setattr(bench, "BATCHED_TRAFFIC_FILE", str(root / "profiles" / "batched.json"))
    sweep = "void rlpt::(anonymous namespace)::k_sweep<float, 256, 2, 0, false>(x)"
    probe = "void rlpt::(anonymous namespace)::k_stream_lists<256>(x)"
    copy = "__amd_rocclr_copyBuffer"
    _csv(str(d / "kt" / "kt_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"],
         [[sweep, 20, 2.5e6, 2.4e6, 2.6e6, 90.0], [probe, 10, 2.4e6, 2.3e6, 2.5e6, 9.0]])
    cc = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy: FETCH_SIZE reads half the copied bytes, WRITE_SIZE all of them
    _csv(str(d / "cal_FETCH_SIZE" / "cal_counter_collection.csv"), cc, [[copy, "FETCH_SIZE", 262144.0]])
    _csv(str(d / "cal_WRITE_SIZE" / "cal_counter_collection.csv"), cc, [[copy, "WRITE_SIZE", 524288.0]])
    _csv(str(d / "pmc_FETCH_SIZE" / "pmc_counter_collection.csv"), cc,
         [[sweep, "FETCH_SIZE", 1000.0], [sweep, "FETCH_SIZE", 3000.0], [probe, "FETCH_SIZE", 1500.0]])
    _csv(str(d / "pmc_WRITE_SIZE" / "pmc_counter_collection.csv"), cc,
         [[sweep, "WRITE_SIZE", 10.0], [sweep, "WRITE_SIZE", 30.0], [probe, "WRITE_SIZE", 0.0]])
    bench.summarize_profiles(str(d))
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_kib_per_dispatch"] == pytest.approx(2000.0) and t["dispatches"] == [2, 2]
    assert t["hbm_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0 + 20.0 * 1024 * 1.0)
    assert t["ceiling_hbm_bytes_per_launch"] == pytest.approx(1500.0 * 1024 * 2.0)
    assert t["avg_duration_ns_kernel_trace"] == pytest.approx(2.5e6)
    assert all(c.startswith("rocprofv3 --pmc ") and "gpurun_out/prof/" in c for c in t["commands"])
    text = open(os.path.join(str(root), "profiles", "sweep_n256_kernel_stats.txt")).read()
    assert "k_sweep<float, 256, 2, 0, false>" in text and "anonymous namespace" not in text
    # the bench takes the committed traffic only while the kernel source is the one it was taken on
    assert bench.traffic_for_current_kernel(1.0, bench.TRAFFIC_FILE) == pytest.approx(t["hbm_bytes_per_launch"])
    t["kernel_source_sha"] = "0" * 16
    json.dump(t, open(bench.TRAFFIC_FILE, "w"))
    assert bench.traffic_for_current_kernel(1.0, bench.TRAFFIC_FILE) is None
