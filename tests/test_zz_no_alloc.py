"""The search entry point that allocates nothing (genie_search_noalloc_async):
its workspace is the device array the library holds per GPU.  Checked
against genie_search_async (caller workspace) and the oracle, bit for bit,
on two calls in a row, the second with fewer queries, fewer tiles and
another k, so that what the first call left in the shared array must not
leak into the second's answers; plus the size limit."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(ix, queries, k):
    off, items = genie.queries_to_device(queries.q_offsets, queries.items)
    mi = max(1, queries.max_items())
    ref_ids, ref_cts, ws = genie.genie_search_async(ix, off, items, k, mi)
    ids = torch.full_like(ref_ids, -7)
    cts = torch.full_like(ref_cts, -7)
    genie.genie_search_noalloc_async(ix, off, items, k, mi, ids, cts)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] == 0
    return (genie.as_uint32(ids), genie.as_uint32(cts), genie.as_uint32(ref_ids),
            genie.as_uint32(ref_cts))


def _oracle(values, V, queries, k):
    o_ids, o_cts, _, _ = oracle.search_idx(oracle.build_csr(values, V), queries, k)
    return o_ids, o_cts


def test_noalloc_matches_workspace_search_twice():
    # first call: 3 full tiles and a ragged fourth, 96 queries, k = 100
    big = workloads.relational(n=3 * 65535 + 777, d=8, V=32, nq=96, k=100)
    print("noalloc call 1:", big.n, "objects,", big.queries.n_queries, "queries, k=100",
          flush=True)
    ix = genie.Index(big.values, big.V)
    ids, cts, r_ids, r_cts = _both(ix, big.queries, 100)
    assert np.array_equal(ids, r_ids) and np.array_equal(cts, r_cts)
    o_ids, o_cts = _oracle(big.values, big.V, big.queries, 100)
    assert np.array_equal(ids, o_ids) and np.array_equal(cts, o_cts)
    ix.free()
    # second call, smaller: 2 tiles (one ragged), 20 queries, k = 7
    small = workloads.tiny(n=70_000, nq=20, k=7)
    print("noalloc call 2:", small.n, "objects,", small.queries.n_queries, "queries, k=7",
          flush=True)
    ix = genie.Index(small.values, small.V)
    ids, cts, r_ids, r_cts = _both(ix, small.queries, 7)
    assert np.array_equal(ids, r_ids) and np.array_equal(cts, r_cts)
    o_ids, o_cts = _oracle(small.values, small.V, small.queries, 7)
    assert np.array_equal(ids, o_ids) and np.array_equal(cts, o_cts)
    ix.free()


def test_noalloc_rejects_oversized_calls():
    inst = workloads.tiny(n=70_000, nq=4, k=10)
    ix = genie.Index(inst.values, inst.V)
    lib = genie.load()
    k = 1000
    # queries whose workspace exceeds the held array: refused before any launch
    nq = genie.NOALLOC_WORKSPACE_BYTES // (ix.info.n_tiles * k * 8) + 1
    assert genie.genie_search_workspace_size(ix, nq, k) > genie.NOALLOC_WORKSPACE_BYTES
    print("noalloc oversize:", nq, "queries at k =", k, flush=True)
    rc = lib.genie_search_noalloc_async(ix.handle, None, None, 0, nq, 16, k, None, None, None)
    assert rc == genie.GENIE_ERANGE
    assert b"held workspace" in lib.genie_last_error()
    # the largest call that fits still runs and is exact
    fit = genie.NOALLOC_WORKSPACE_BYTES // (ix.info.n_tiles * k * 8) - 64
    assert genie.genie_search_workspace_size(ix, fit, k) <= genie.NOALLOC_WORKSPACE_BYTES
    qs = workloads.queries_halfwidth(np.random.default_rng(5), inst.values, inst.V, fit, 2)
    print("noalloc largest fitting call:", fit, "queries at k =", k, flush=True)
    ids, cts, r_ids, r_cts = _both(ix, qs, k)
    assert np.array_equal(ids, r_ids) and np.array_equal(cts, r_cts)
    ix.free()
