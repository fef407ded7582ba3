"""CPU checks of the library: it loads, exports every declared symbol, and its
host graph builder and analysis helpers agree with the oracle."""
import math
import os
import re

import numpy as np
import pytest

from paper_2511_13508_amd import rlpt
from tests import brute

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rlpt.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(rlpt_\w+)\s*\(", text, re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    L = rlpt.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(rlpt.EXPORTS) == names
    assert rlpt.abi_version() == 1


@pytest.mark.parametrize("N,seed,kind,mask", [
    (4, 0, rlpt.OMEGA_COMB, rlpt.SPLIT_ALL), (5, 0, rlpt.OMEGA_COMB, rlpt.SPLIT_ALL),
    (16, 1, rlpt.OMEGA_RANDOM, rlpt.SPLIT_ALL), (17, 2, rlpt.OMEGA_RANDOM, rlpt.SPLIT_ALL),
    (32, 3, rlpt.OMEGA_RANDOM, rlpt.SPLIT_A), (48, 4, rlpt.OMEGA_RANDOM, rlpt.SPLIT_ALL),
    (64, 2511135081, rlpt.OMEGA_RANDOM, rlpt.SPLIT_ALL), (40, 5, rlpt.OMEGA_COMB, rlpt.SPLIT_ALL),
])
def test_graph_builder_matches_oracle(oracle, N, seed, kind, mask):
    g = rlpt.Graph(N, seed, kind, mask)
    omega, quads, J = g.export()
    go = oracle.Graph(N, seed, kind, mask)
    assert np.array_equal(omega, go.omega)
    assert np.array_equal(quads, go.quads)
    np.testing.assert_allclose(J, go.J, rtol=1e-15, atol=0)
    info = g.info()
    assert info["n_terms"] == go.n_terms
    assert info["deg_sum"] == 4 * go.n_terms
    assert info["sigma2"] == pytest.approx(N / go.n_terms, rel=1e-15)
    deg = np.bincount(go.quads.astype(np.int64).ravel(), minlength=N)
    assert info["deg_min"] == deg.min() and info["deg_max"] == deg.max()
    assert info["list_entries"] == int(np.sum((deg + 3) // 4 * 4))


def test_graph_builder_large_n_count(oracle):
    """N = 128 (by-pair-sum window search) against the oracle's four-fold loop."""
    g = rlpt.Graph(128, 77)
    go = oracle.Graph(128, 77)
    _, quads, J = g.export()
    assert np.array_equal(quads, go.quads)
    np.testing.assert_allclose(J, go.J, rtol=1e-15)


def test_graph_builder_rejects_bad_input():
    with pytest.raises(rlpt.RlptError) as e:
        rlpt.Graph(3, 0)
    assert e.value.code == rlpt.RLPT_E_ARG
    with pytest.raises(rlpt.RlptError):
        rlpt.Graph(2000, 0)
    with pytest.raises(rlpt.RlptError):
        rlpt.Graph(16, 0, split_mask=0)


def test_comb_closed_form_from_library():
    for N in (8, 9, 30, 31):
        assert rlpt.Graph(N, 0, rlpt.OMEGA_COMB).info()["n_terms"] == brute.comb_count(N)


def ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / math.sqrt(1 - phi ** 2)
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    return x


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_tau_int_ar1_closed_form_and_oracle(phi):
    from oracle import analysis
    x = ar1(phi, 20000, 3)
    exact = (1 + phi) / (2 * (1 - phi))
    t_or, w_or = analysis.tau_int(x)
    t_lib, w_lib = rlpt.tau_int(x)
    assert t_or == pytest.approx(exact, rel=0.15)
    assert t_lib == pytest.approx(t_or, rel=1e-10)
    assert w_lib == w_or


def test_jackknife_of_mean_is_standard_error():
    from oracle import analysis
    rng = np.random.default_rng(1)
    v = rng.standard_normal((50, 3))
    m, e = analysis.jackknife_mean_err(v)
    np.testing.assert_allclose(m, v.mean(0))
    np.testing.assert_allclose(e, v.std(0, ddof=1) / math.sqrt(50), rtol=1e-12)


def test_tune_registry_roundtrip(tmp_path):
    rlpt.tune_clear()
    rlpt.tune_set(64, rlpt.FP32, 0, 256, 4, 1.5)
    rlpt.tune_set(64, rlpt.FP32, 0, 256, 4, 1.25)  # same key: replaced
    rlpt.tune_set(128, rlpt.FP32, 0, 512, 2, 3.0)
    assert len(rlpt.tune_entries()) == 2
    p = str(tmp_path / "tiles.jsonl")
    rlpt.tune_save(p)
    rlpt.tune_clear()
    assert rlpt.tune_entries() == []
    rlpt.tune_load(p)
    e = sorted(rlpt.tune_entries(), key=lambda d: d["n_modes"])
    assert [(d["n_modes"], d["block_threads"], d["copies_per_block"]) for d in e] == [(64, 256, 4), (128, 512, 2)]
    assert e[0]["ms_per_sweep"] == pytest.approx(1.25)
    with pytest.raises(rlpt.RlptError):
        rlpt.tune_set(64, rlpt.FP32, 0, 100, 1, 1.0)  # not a power of two
    with pytest.raises(rlpt.RlptError):
        rlpt.tune_set(64, rlpt.FP32, 0, 128, 4, 1.0)  # more copies than waves
    rlpt.tune_clear()
