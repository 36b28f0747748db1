"""Pins of the oracle's ANN quality measures (Section 6.4.1): exact k nearest
neighbours under l2 and l1, recall, and the approximation ratio.

Nothing here runs on the GPU.  The neighbours are pinned by hand-worked
2-D and 3-D cases with ties (the order is distance ascending, then id
ascending) and by a brute-force sort of directly computed distances on
random integer points, where every distance is exact in float64 so that
ties are exact on both sides.  Recall and the approximation ratio are pinned
by hand-worked values; the ratio follows the section's formula (the mean
over i of the i-th returned distance over the i-th true distance, both lists
sorted ascending), skipping a pair whose true distance is zero.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import rbh

# 2-D points: small integers, so squared distances are exact in float64
P2 = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 0], [3, 4]], dtype=np.float32)


def test_l2_hand_worked_2d_with_ties():
    q = np.array([[0, 0], [1, 0.5]], dtype=np.float32)
    ids, dist = oracle.exact_knn_l2(P2, q, 4)
    # from (0, 0): p0 at 0, p1 and p2 at 1 (tie: lower id first), p3 at sqrt 2
    assert ids[0].tolist() == [0, 1, 2, 3]
    assert np.allclose(dist[0], [0.0, 1.0, 1.0, math.sqrt(2.0)], rtol=0, atol=1e-12)
    # from (1, 0.5): p1 and p3 at 0.5, then p0, p2, p4 all at sqrt(1.25)
    assert ids[1].tolist() == [1, 3, 0, 2]
    assert np.allclose(dist[1], [0.5, 0.5, math.sqrt(1.25), math.sqrt(1.25)], rtol=0,
                       atol=1e-12)
    ids6, _ = oracle.exact_knn_l2(P2, q[1:], 6)
    assert ids6[0].tolist() == [1, 3, 0, 2, 4, 5]


def test_l2_hand_worked_3d():
    P = np.array([[1, 1, 1], [0, 0, 0], [2, 2, 2], [1, 1, 3], [3, 1, 1], [1, 2, 1]],
                 dtype=np.float32)
    q = np.array([[1, 1, 1]], dtype=np.float32)
    ids, dist = oracle.exact_knn_l2(P, q, 6)
    # distances: 0, sqrt3, sqrt3, 2, 2, 1
    assert ids[0].tolist() == [0, 5, 1, 2, 3, 4]
    want = [0.0, 1.0, math.sqrt(3.0), math.sqrt(3.0), 2.0, 2.0]
    assert np.allclose(dist[0], want, rtol=0, atol=1e-12)


def test_l1_hand_worked_2d_and_3d_with_ties():
    ids, dist = rbh.exact_knn_l1(P2, np.array([[1, 0.5]], dtype=np.float32), 6)
    # |dx| + |dy|: p0 1.5, p1 0.5, p2 1.5, p3 0.5, p4 1.5, p5 5.5
    assert ids[0].tolist() == [1, 3, 0, 2, 4, 5]
    assert np.allclose(dist[0], [0.5, 0.5, 1.5, 1.5, 1.5, 5.5], rtol=0, atol=0)
    P = np.array([[1, 1, 1], [0, 0, 0], [2, 2, 2], [1, 1, 3], [3, 1, 1], [1, 2, 1]],
                 dtype=np.float32)
    ids, dist = rbh.exact_knn_l1(P, np.array([[1, 1, 1]], dtype=np.float32), 6)
    # l1: 0, 3, 3, 2, 2, 1 -- unlike l2, p3 and p4 come before p1 and p2
    assert ids[0].tolist() == [0, 5, 3, 4, 1, 2]
    assert dist[0].tolist() == [0.0, 1.0, 2.0, 2.0, 3.0, 3.0]


@pytest.mark.parametrize("norm", ["l2", "l1"])
def test_knn_equals_brute_force_sort(norm):
    rng = np.random.default_rng(11)
    for trial in range(20):
        n, dim = int(rng.integers(1, 60)), int(rng.integers(1, 5))
        P = rng.integers(-3, 4, size=(n, dim)).astype(np.float32)   # many exact ties
        Q = rng.integers(-3, 4, size=(4, dim)).astype(np.float32)
        k = int(rng.integers(1, n + 1))
        if norm == "l2":
            ids, dist = oracle.exact_knn_l2(P, Q, k)
        else:
            ids, dist = rbh.exact_knn_l1(P, Q, k)
        for r, q in enumerate(Q):
            if norm == "l2":
                d = [math.sqrt(sum((float(a) - float(b)) ** 2 for a, b in zip(p, q))) for p in P]
            else:
                d = [sum(abs(float(a) - float(b)) for a, b in zip(p, q)) for p in P]
            order = sorted(range(n), key=lambda i: (d[i], i))[:k]
            assert ids[r].tolist() == order, (trial, r)
            assert np.allclose(dist[r], [d[i] for i in order], rtol=0, atol=1e-12)


def test_recall_hand_worked():
    found = np.array([[1, 2, 3], [4, 5, 6]])
    true = np.array([[1, 2, 9], [6, 5, 4]])
    assert oracle.recall(found, true) == pytest.approx(5 / 6, abs=0)
    assert oracle.recall(true, true) == 1.0
    assert oracle.recall(np.array([[7, 8, 9]]), np.array([[1, 2, 3]])) == 0.0


def test_approximation_ratio_hand_worked():
    # points on the x axis at 1, 2, 3, 4 from the query at the origin
    P = np.array([[1, 0], [2, 0], [3, 0], [4, 0]], dtype=np.float32)
    q = np.array([[0, 0]], dtype=np.float32)
    true_d = np.array([[1.0, 2.0]])
    # returned {p2, p1} (distances 3 and 2, in that order): sorted 2, 3 against
    # 1, 2 -> (2/1 + 3/2) / 2 = 1.75
    assert oracle.approximation_ratio(P, q, np.array([[2, 1]]), true_d) == pytest.approx(1.75)
    # the true neighbours themselves: 1
    assert oracle.approximation_ratio(P, q, np.array([[1, 0]]), true_d) == pytest.approx(1.0)
    # two queries: the mean of their ratios
    q2 = np.array([[0, 0], [5, 0]], dtype=np.float32)
    td2 = np.array([[1.0, 2.0], [1.0, 2.0]])
    got = oracle.approximation_ratio(P, q2, np.array([[3, 2], [3, 2]]), td2)
    # query 1: found at 4, 3 -> sorted 3, 4 -> (3 + 2) / 2 = 2.5; query 2: found
    # at 1, 2 -> (1 + 1) / 2 = 1
    assert got == pytest.approx((2.5 + 1.0) / 2)
    # a zero true distance is skipped: true 0, 1; found at 1, 2 -> 2 / 1
    P0 = np.array([[0, 0], [1, 0], [2, 0]], dtype=np.float32)
    assert oracle.approximation_ratio(P0, q, np.array([[1, 2]]),
                                      np.array([[0.0, 1.0]])) == pytest.approx(2.0)


def test_approximation_ratio_on_exact_neighbours_is_one():
    rng = np.random.default_rng(5)
    P = rng.standard_normal((300, 6)).astype(np.float32)
    Q = rng.standard_normal((7, 6)).astype(np.float32)
    ids, dist = oracle.exact_knn_l2(P, Q, 10)
    assert oracle.approximation_ratio(P, Q, ids, dist) == pytest.approx(1.0, abs=1e-12)
    # any other 10 points are at least as far, rank by rank
    worse = (ids + 1) % 300
    assert oracle.approximation_ratio(P, Q, worse, dist) >= 1.0
