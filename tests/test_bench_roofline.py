"""The bench line's roofline logic on the host: which roof binds and what
its fraction is, for launches shaped like the workloads' (no GPU)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PEAKS = {"lds_atomic_conflict_free": 9.5e12, "lds_atomic_random": 5.4e12,
         "lds_atomic_one_bank_per_lane": 9.5e12}


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_cache_served_index_binds_on_lds_atomics(bench):
    # 5.68 G postings in 1.4 ms: 4 B per posting would need 16 TB/s of HBM,
    # and the counters saw 0.42 GB; the atomics bind
    r = bench.roofs(5_680_000_000, 32 * 1024, 1024, 100, 16, 1.4, PEAKS, 420_000_000)
    assert r["bound"] == "lds_atomic"
    assert r["frac"] == pytest.approx(5.68e9 / 1.4e-3 / 9.5e12, rel=1e-3)
    assert r["hbm_alg_frac"] > 1.0


def test_streamed_index_binds_on_measured_hbm(bench):
    # algorithmic bytes above HBM's rate, measured traffic 70 GB in 12 ms:
    # HBM binds, priced in the measured bytes, and stays under its peak
    r = bench.roofs(44_000_000_000, 237 * 4096, 4096, 100, 16, 12.0, PEAKS, 70_000_000_000)
    assert r["bound"] == "hbm"
    assert r["achieved"] == pytest.approx(70e9 / 12e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(70e9 / 12e-3 / 8e12, rel=1e-3)
    assert 0 < r["frac"] <= 1.0 and "measured" in r["achieved_bytes"]


def test_measured_traffic_below_the_atomic_fraction_does_not_bind(bench):
    # algorithmic bytes under HBM's peak, but the counters saw little HBM
    # traffic: the atomics bind (a cache-served short-run workload)
    r = bench.roofs(7_560_000_000, 38 * 1024, 1024, 32, 77, 4.03, PEAKS, 1_270_000_000)
    assert r["hbm_alg_frac"] <= 1.0
    assert r["bound"] == "lds_atomic"


def test_without_counters_algorithmic_bytes_decide(bench):
    # a launch-bound tiny batch, no counter summary: HBM in algorithmic bytes
    r = bench.roofs(1_230_000, 1600, 100, 10, 1, 0.018, PEAKS, None)
    assert r["bound"] == "hbm" and r["achieved_bytes"] == "algorithmic"
    alg = 4 * 1_230_000 + 28 * 1600 + 8 * 10 * 100
    assert r["hbm_alg_bytes_per_launch"] == alg
    assert r["frac"] == pytest.approx(alg / 0.018e-3 / 8e12, rel=1e-3)
    # and algorithmic bytes above the peak never make HBM the bound
    r = bench.roofs(5_680_000_000, 32 * 1024, 1024, 100, 16, 1.4, PEAKS, None)
    assert r["bound"] == "lds_atomic"
