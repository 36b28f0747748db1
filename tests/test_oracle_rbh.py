"""Pins of the RBH / MurmurHash3 oracle (Section 4.1.3) against things other
than itself: scikit-learn's independent MurmurHash3_x86_32, a hand-worked
binning, the collision probability the construction must have (the
Laplacian kernel), and the spread of the re-hash."""
import numpy as np
import pytest

from oracle import rbh

sklearn_murmur = pytest.importorskip("sklearn.utils").murmurhash3_32


def test_murmur3_matches_an_independent_implementation():
    rng = np.random.default_rng(0)
    for L in (1, 2, 3, 4, 7, 16, 33, 128):
        for seed in (0, 1, 12345, 2**31 + 7, 0xFFFFFFFF):
            w = rng.integers(0, 2**32, size=(6, L), dtype=np.uint64).astype(np.uint32)
            mine = rbh.murmur3_32_words(w, seed)
            for r in range(6):
                assert int(mine[r]) == sklearn_murmur(w[r].tobytes(), seed=seed, positive=True)


def test_hand_worked_bins_and_bucket():
    p = np.array([[1.5, -0.2, 3.0]])
    g = np.array([[0.5, 2.0, 1.0]])
    u = np.array([[0.3, 0.1, 0.0]])
    # (1.5-0.3)/0.5 = 2.4 -> 2; (-0.2-0.1)/2 = -0.15 -> -1; 3/1 = 3 -> 3
    assert rbh.rbh_bins_f64(p, g, u).tolist() == [[[2, -1, 3]]]
    key = np.array([2, -1, 3], dtype="<i4").tobytes()
    want = sklearn_murmur(key, seed=7, positive=True) >> (32 - 13)
    got = rbh.rbh_signatures(p, g, u, np.array([7], np.uint32), 13)
    assert int(got[0, 0]) == want


def test_collision_probability_is_the_laplacian_kernel():
    rng = np.random.default_rng(5)
    sigma, N = 2.0, 200_000
    p = np.array([0.3, 1.1, -0.4, 2.0])
    for delta in ([0.5, 1.0, 2.0, 0.25], [0.1, 0.0, 0.3, 0.05], [0.0, 0.0, 0.0, 0.0]):
        q = p + np.array(delta)
        g = rng.gamma(2.0, sigma, size=(N, 4))
        u = rng.random((N, 4)) * g
        bp = rbh.rbh_bins_f64(p[None], g, u)[0]
        bq = rbh.rbh_bins_f64(q[None], g, u)[0]
        rate = np.mean((bp == bq).all(axis=1))
        want = float(rbh.laplacian_kernel(p, q, sigma))
        se = np.sqrt(max(want * (1 - want), 1e-12) / N)
        assert abs(rate - want) <= 4 * se + 1e-12, (delta, rate, want)


def test_rehash_spreads_distinct_bins_uniformly():
    rng = np.random.default_rng(9)
    words = rng.integers(-50, 50, size=(60_000, 8)).astype(np.int32).view(np.uint32)
    words = np.unique(words, axis=0)
    b = rbh.murmur3_32_words(words, 99) >> np.uint32(32 - 8)
    counts = np.bincount(b.astype(np.int64), minlength=256)
    expected = len(words) / 256
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 255 degrees of freedom: mean 255, sd ~ 22.6; a loose 6-sigma bound
    assert chi2 < 255 + 6 * 22.6
