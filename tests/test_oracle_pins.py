"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here runs on the GPU.  Each test ties the oracle to something other
than itself: the paper's worked values, a set-theoretic brute force of
Definition 2.1 on tiny inputs, invariants, special cases with a known answer,
and the two proved properties of c-PQ (Lemma 3.1, Theorem 3.1).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fig1():
    with open(os.path.join(GOLD, "fig1_cpq_example.json")) as f:
        return json.load(f)


def _queries(items_list):
    lens = [len(x) for x in items_list]
    off = np.zeros(len(lens) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens)
    items = (np.concatenate([np.asarray(x, dtype=np.uint32).reshape(-1, 3) for x in items_list])
             if sum(lens) else np.zeros((0, 3), dtype=np.uint32))
    return workloads.Queries(off, items.reshape(-1, 3))


# ---------------------------------------------------------------------------
# Definition 2.1: the paper's worked value
# ---------------------------------------------------------------------------

def test_definition_worked_value():
    g = _fig1()
    values = np.array(g["objects"], dtype=np.uint32)
    items = np.array(g["query"], dtype=np.uint32)
    per_item = [int(oracle.brute_force_counts(values[:1], items[i:i + 1])[0]) for i in range(3)]
    assert per_item == g["c_items_o1"]
    assert int(oracle.brute_force_counts(values, items)[0]) == g["mc_q1_o1"]
    idx = oracle.build_csr(values, g["V"])
    counts, scanned = oracle.match_counts(idx, items)
    assert int(counts[0]) == g["mc_q1_o1"]
    assert scanned == int(counts.sum())


def _set_brute_force(values, items):
    """Definition 2.1 read literally on sets: O = {(j, v_j)}, item r = the set
    {(dim, v) : lo <= v <= hi}; C(r, O) = |O intersect r|."""
    out = []
    for row in values:
        obj = {(j, int(v)) for j, v in enumerate(row)}
        mc = 0
        for dim, lo, hi in items:
            r = {(int(dim), v) for v in range(int(lo), int(hi) + 1)}
            mc += len(obj & r)
        out.append(mc)
    return np.array(out, dtype=np.int64)


def test_brute_force_matches_set_definition():
    rng = np.random.default_rng(7)
    for trial in range(40):
        n, d, V = int(rng.integers(1, 12)), int(rng.integers(1, 4)), int(rng.integers(1, 6))
        inst = workloads.random_small(rng, n, d, V, 3, 6)
        for q in range(inst.queries.n_queries):
            items = inst.queries.items_of(q)
            a = oracle.brute_force_counts(inst.values, items)
            b = _set_brute_force(inst.values, items)
            assert np.array_equal(a, b), (trial, q, items)


# ---------------------------------------------------------------------------
# O1 (definition) == O2 (index scan) on random tiny inputs, every k
# ---------------------------------------------------------------------------

def test_index_scan_equals_brute_force_tiny():
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(1, 65))
        d = int(rng.integers(1, 5))
        V = int(rng.integers(1, 9))
        inst = workloads.random_small(rng, n, d, V, 6, 8)
        idx = oracle.build_csr(inst.values, V)
        for k in range(1, n + 3):
            ids2, cts2, kth2, scanned = oracle.search_idx(idx, inst.queries, k)
            ids1, cts1 = oracle.brute_force_topk(inst.values, inst.queries, k)
            assert np.array_equal(ids1, ids2), (trial, k)
            assert np.array_equal(cts1, cts2), (trial, k)
            for q in range(inst.queries.n_queries):
                counts = oracle.brute_force_counts(inst.values, inst.queries.items_of(q))
                # posting-sum invariant: each scanned posting adds exactly one
                assert int(scanned[q]) == int(counts.sum())
                if n >= k:
                    assert int(kth2[q]) == int(np.sort(counts)[::-1][k - 1])


def test_total_order_by_permutation_brute_force():
    """For n <= 6 the answer equals the first k of the lexicographic minimum
    over all permutations of (-count, id): a textbook definition of the order."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(1, 7))
        inst = workloads.random_small(rng, n, 2, 3, 2, 4)
        idx = oracle.build_csr(inst.values, 3)
        for q in range(inst.queries.n_queries):
            counts = oracle.brute_force_counts(inst.values, inst.queries.items_of(q))
            best = min(itertools.permutations(range(n)),
                       key=lambda p: [(-counts[i], i) for i in p])
            for k in (1, 2, n, n + 1):
                ids, cts, _, _ = oracle.search_idx(idx, inst.queries, k, q, q + 1)
                want = list(best[:min(k, n)]) + [oracle.UINT32_MAX] * max(0, k - n)
                assert [int(x) for x in ids[0]] == want


# ---------------------------------------------------------------------------
# special cases with a known answer
# ---------------------------------------------------------------------------

def test_identical_objects_give_first_ids():
    values = np.full((50, 4), 3, dtype=np.uint32)
    qs = _queries([[[0, 2, 4], [1, 3, 3], [2, 0, 1], [3, 3, 9]]])
    idx = oracle.build_csr(values, 8)
    ids, cts, kth, _ = oracle.search_idx(idx, qs, 7)
    assert list(ids[0]) == list(range(7))
    assert list(cts[0]) == [3] * 7
    assert int(kth[0]) == 3


def test_full_range_items_count_every_object():
    rng = np.random.default_rng(5)
    values = rng.integers(0, 16, size=(200, 5), dtype=np.uint32)
    qs = _queries([[[j, 0, 15] for j in range(5)] + [[2, 0, 100]]])
    idx = oracle.build_csr(values, 16)
    counts, scanned = oracle.match_counts(idx, qs.items_of(0))
    assert np.all(counts == 6)
    assert scanned == 200 * 6


def test_empty_query_and_empty_items():
    values = np.arange(30, dtype=np.uint32).reshape(10, 3) % 7
    qs = _queries([[], [[0, 5, 2], [1, 9, 20]]])
    idx = oracle.build_csr(values, 7)
    ids, cts, kth, scanned = oracle.search_idx(idx, qs, 4)
    for q in range(2):
        assert list(ids[q]) == [0, 1, 2, 3]
        assert list(cts[q]) == [0, 0, 0, 0]
        assert int(scanned[q]) == 0


def test_k_larger_than_n_pads():
    values = np.array([[0], [1], [1]], dtype=np.uint32)
    qs = _queries([[[0, 1, 1]]])
    idx = oracle.build_csr(values, 2)
    ids, cts, kth, _ = oracle.search_idx(idx, qs, 5)
    assert list(ids[0]) == [1, 2, 0, oracle.UINT32_MAX, oracle.UINT32_MAX]
    assert list(cts[0]) == [1, 1, 0, 0, 0]
    assert int(kth[0]) == 0


def test_own_values_rank_first():
    """An exact-match query on object o's own values gives o the largest
    possible count d; it ranks first unless a smaller id has the same row."""
    rng = np.random.default_rng(9)
    values = rng.integers(0, 5, size=(300, 6), dtype=np.uint32)
    idx = oracle.build_csr(values, 5)
    for o in rng.integers(0, 300, size=10):
        qs = _queries([[[j, int(values[o, j]), int(values[o, j])] for j in range(6)]])
        ids, cts, _, _ = oracle.search_idx(idx, qs, 3)
        first = int(np.nonzero((values == values[o]).all(axis=1))[0][0])
        assert int(ids[0, 0]) == first and int(cts[0, 0]) == 6


def test_widening_never_lowers_counts():
    rng = np.random.default_rng(12)
    inst = workloads.tiny(n=2000, nq=5)
    idx = oracle.build_csr(inst.values, inst.V)
    for q in range(5):
        items = inst.queries.items_of(q).astype(np.int64)
        wide = items.copy()
        wide[:, 1] = np.maximum(0, wide[:, 1] - rng.integers(0, 3, size=len(wide)))
        wide[:, 2] = wide[:, 2] + rng.integers(0, 3, size=len(wide))
        a, _ = oracle.match_counts(idx, items.astype(np.uint32))
        b, _ = oracle.match_counts(idx, wide.astype(np.uint32))
        assert np.all(b >= a)


def test_invalid_dim_is_rejected():
    values = np.zeros((4, 2), dtype=np.uint32)
    idx = oracle.build_csr(values, 3)
    with pytest.raises(ValueError):
        oracle.search_idx(idx, _queries([[[2, 0, 1]]]), 1)


def test_csr_lists_ascending_and_complete():
    inst = workloads.relational(n=5000, d=4, V=16, nq=1)
    idx = oracle.build_csr(inst.values, inst.V)
    for j in range(4):
        for v in range(16):
            p = idx.postings(j, v)
            assert np.all(np.diff(p.astype(np.int64)) > 0)
            assert np.array_equal(p, np.nonzero(inst.values[:, j] == v)[0].astype(np.uint32))


# ---------------------------------------------------------------------------
# c-PQ (Algorithm 1): the worked example and the proved properties
# ---------------------------------------------------------------------------

def test_cpq_worked_example_trace():
    g = _fig1()
    values = np.array(g["objects"], dtype=np.uint32)
    idx = oracle.build_csr(values, g["V"])
    tr = oracle.cpq_simulate(idx, np.array(g["query"], dtype=np.uint32), g["k"])
    assert len(tr.steps) == 3
    for got, want in zip(tr.steps, g["trace"]):
        assert got["bc"] == {int(a): b for a, b in want["bc"].items()}
        assert got["ht"] == {int(a): b for a, b in want["ht"].items()}
        assert got["za"] == want["za"]
        assert got["at"] == want["at"]
    # Theorem 3.1: MC_k = AT - 1, and the top-1 is in the HT
    assert tr.at - 1 == g["top1"]["count"]
    assert tr.ht[g["top1"]["id"]] == g["top1"]["count"]
    ids, cts, _, _ = oracle.search_idx(idx, _queries([g["query"]]), 1)
    assert int(ids[0, 0]) == g["top1"]["id"] and int(cts[0, 0]) == g["top1"]["count"]


def _check_cpq_properties(idx, items, k, counts):
    tr = oracle.cpq_simulate(idx, items, k)
    za, at = tr.za, tr.at
    n = len(counts)
    # Lemma 3.1: ZA[AT] < k and (when AT > 1) ZA[AT-1] >= k
    assert za[at] < k
    if at > 1:
        assert za[at - 1] >= k
    # Theorem 3.1: MC_k = AT - 1 (k-th count of the total order, 0-counts
    # included, provided n >= k)
    if n >= k:
        kth = int(np.sort(counts)[::-1][k - 1])
        assert at - 1 == kth
    # every object with count >= AT is in the HT with its exact count
    for o in np.nonzero(counts >= at)[0]:
        assert tr.ht.get(int(o)) == int(counts[o])
    # HT entries never exceed the true count
    for o, v in tr.ht.items():
        assert v <= counts[o]
    # size bound O(k * AT): first entry of an object happens only at level AT,
    # at most k times per level
    assert len(tr.ht) <= k * at
    return tr


def test_cpq_properties_random_tiny():
    rng = np.random.default_rng(21)
    for trial in range(80):
        n = int(rng.integers(1, 40))
        d = int(rng.integers(1, 5))
        V = int(rng.integers(1, 6))
        inst = workloads.random_small(rng, n, d, V, 4, 10)
        idx = oracle.build_csr(inst.values, V)
        for q in range(inst.queries.n_queries):
            items = inst.queries.items_of(q)
            counts = oracle.brute_force_counts(inst.values, items)
            for k in (1, 2, 3, max(1, n // 2), n, n + 1):
                _check_cpq_properties(idx, items, k, counts)


def test_cpq_properties_tiny_workload():
    inst = workloads.tiny(nq=20)
    idx = oracle.build_csr(inst.values, inst.V)
    for q in range(20):
        items = inst.queries.items_of(q)
        counts = oracle.brute_force_counts(inst.values, items)
        _check_cpq_properties(idx, items, inst.k, counts)


def test_ht_only_selection_can_miss_ties():
    """The HT need not hold every object tied at the k-th count: an object
    reaching AT-1 after AT moved past it is never inserted at that value.
    This is why exact (count desc, id asc) answers read tied counts from the
    counters, not from the HT."""
    inst = workloads.tiny(nq=40)
    idx = oracle.build_csr(inst.values, inst.V)
    missed = 0
    for q in range(40):
        items = inst.queries.items_of(q)
        counts = oracle.brute_force_counts(inst.values, items)
        tr = oracle.cpq_simulate(idx, items, inst.k)
        ties = set(np.nonzero(counts == tr.at - 1)[0].tolist())
        in_ht = {o for o, v in tr.ht.items() if v == tr.at - 1}
        missed += len(ties - in_ht) > 0
    assert missed > 0
