"""Multiple loadings (Section 3.4) on the GPU: an index cut into parts that
stream through two device slots gives, bit for bit, the answers of the
oracle over all the objects, whatever the part size (aligned to tiles or
not), the tiling, the counter width, k > n, and on repeated calls."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402

pytestmark = pytest.mark.gpu


def _check_parts(values, V, queries, k, part_objects, tile_log2=16, reps=1):
    print("parts", values.shape, part_objects, tile_log2, k, flush=True)
    parts = genie.PartsIndex(values, V, part_objects, tile_log2)
    n = values.shape[0]
    assert parts.info["n_parts"] == (n + part_objects - 1) // part_objects
    off, items = genie.queries_to_device(queries.q_offsets, queries.items)
    o_ids, o_cts, _, scanned = oracle.search_idx(oracle.build_csr(values, V), queries, k)
    ws = parts.workspace(queries.n_queries, k)
    for _ in range(reps):
        ids, cts, ws = genie.genie_parts_search_async(parts, off, items, k,
                                                      max(1, queries.max_items()), workspace=ws)
        torch.cuda.synchronize()
        st = genie.workspace_stats(ws)
        assert st["status"] == 0
        assert st["postings_scanned"] == int(scanned.sum())
        assert np.array_equal(genie.as_uint32(ids), o_ids)
        assert np.array_equal(genie.as_uint32(cts), o_cts)
    parts.free()


def test_parts_aligned_to_tiles():
    inst = workloads.relational(n=5 * 65535 + 123, d=20, V=40, nq=40, k=100)
    _check_parts(inst.values, inst.V, inst.queries, 100, 2 * 65535, reps=3)


def test_parts_not_aligned_and_smaller_tiles():
    inst = workloads.relational(n=310_000, d=12, V=48, nq=30, k=50)
    _check_parts(inst.values, inst.V, inst.queries, 50, 100_000)
    _check_parts(inst.values, inst.V, inst.queries, 50, 77_777, tile_log2=15)


def test_parts_wide_counters_and_k_above_n():
    inst = workloads.uneven(n=150_000, d=16, V=64, nq=12, smin=200, smax=400)
    _check_parts(inst.values, inst.V, inst.queries, 100, 60_000)
    small = workloads.relational(n=900, d=6, V=10, nq=8, k=1000)
    _check_parts(small.values, small.V, small.queries, 1000, 400)


def test_one_part_equals_one_index():
    inst = workloads.relational(n=2 * 65535 + 9, d=16, V=32, nq=24, k=30)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    ix = genie.Index(inst.values, inst.V)
    a_ids, a_cts, _ = genie.genie_search_async(ix, off, items, 30, inst.queries.max_items())
    parts = genie.PartsIndex(inst.values, inst.V, 10 ** 9)
    b_ids, b_cts, _ = genie.genie_parts_search_async(parts, off, items, 30,
                                                     inst.queries.max_items())
    torch.cuda.synchronize()
    assert parts.info["n_parts"] == 1
    assert torch.equal(a_ids, b_ids) and torch.equal(a_cts, b_cts)
    parts.free()
    ix.free()
