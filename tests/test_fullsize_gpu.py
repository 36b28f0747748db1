"""Full-size workloads on the GPU, checked on sampled rows against the oracle.

* tau-ANN: 1,000,000 points x 128 (Gaussian mixture), 237 E2LSH functions
  re-hashed into 8,192 buckets, 4,096 queries; float64 oracle signatures feed
  both sides, so the match counts are exact.  Recall@100 and the
  approximation ratio against exact l2 are printed (quality, not parity).
* uneven: 10,000,000 objects x 64 dims, 1,024 buckets, Zipf(1.1); queries
  with 4..512 items in one launch (1,024 of the 16,384 of the full batch).
"""
import time

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _check_rows(ix, values, V, queries, k, rows):
    off, items = genie.queries_to_device(queries.q_offsets, queries.items)
    t0 = time.time()
    ids, cts, ws = genie.genie_search_async(ix, off, items, k, queries.max_items())
    torch.cuda.synchronize()
    _log("gpu search", queries.n_queries, "queries", round(time.time() - t0, 2), "s",
         genie.workspace_stats(ws))
    ids, cts = genie.as_uint32(ids), genie.as_uint32(cts)
    oidx = oracle.build_csr(values, V)
    for q in rows:
        o_ids, o_cts, _, _ = oracle.search_idx(oidx, queries, k, q, q + 1)
        assert np.array_equal(ids[q], o_ids[0]), q
        assert np.array_equal(cts[q], o_cts[0]), q
    _log("checked rows", list(rows))
    return ids


def test_ann_full_size_sampled():
    t0 = time.time()
    inp = workloads.ann()
    sig = oracle.lsh_signatures(inp.points, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    qsig = oracle.lsh_signatures(inp.queries, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    _log("signatures", round(time.time() - t0, 1), "s")
    q = workloads.queries_exact(qsig)
    ix = genie.Index(sig, 1 << inp.log2_buckets)
    rng = np.random.default_rng(3)
    rows = sorted(rng.choice(q.n_queries, size=12, replace=False).tolist())
    ids = _check_rows(ix, sig, 1 << inp.log2_buckets, q, inp.k, rows)
    ix.free()
    sample = rows + list(range(20))
    t_ids, t_dist = oracle.exact_knn_l2(inp.points, inp.queries[sample], inp.k)
    rec = oracle.recall(ids[sample].astype(np.int64), t_ids)
    ratio = oracle.approximation_ratio(inp.points, inp.queries[sample],
                                       ids[sample].astype(np.int64), t_dist)
    _log("recall@100", round(rec, 4), "approximation ratio", round(ratio, 4))
    assert 0.0 < rec <= 1.0 and ratio >= 1.0


def test_uneven_full_objects_sampled():
    t0 = time.time()
    inst = workloads.uneven(nq=1024)
    _log("generated", round(time.time() - t0, 1), "s")
    ix = genie.Index(inst.values, inst.V)
    _log("index built", round(time.time() - t0, 1), "s", ix.info)
    lens = np.diff(inst.queries.q_offsets.astype(np.int64))
    rows = sorted({int(np.argmin(lens)), int(np.argmax(lens)), 0, 511, 1023})
    _check_rows(ix, inst.values, inst.V, inst.queries, inst.k, rows)
    ix.free()
