"""The Hash Table overflow fallback of the c-PQ (Section 3.3.2: the table is
sized only as O(k x largest count)).  With the table capped far below what
the tiles need, every tile that runs out of slots flags the overflow and
selects from its exact counters; the answers must stay identical to the
oracle on the plain path (one workgroup per pair and persistent), on the
gated path (including queries that fall back to AT = 1) and on the row-count
entry point used for graph replay."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    # 3 full tiles and a ragged fourth; k = 100 needs far more than 4 slots
    inst = workloads.relational(n=3 * 65535 + 2345, d=12, V=48, nq=64, k=100)
    o_ids, o_cts, o_kth, _ = oracle.search_idx(oracle.build_csr(inst.values, inst.V),
                                               inst.queries, inst.k)
    ix = genie.Index(inst.values, inst.V)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    yield inst, ix, off, items, o_ids, o_cts, o_kth
    ix.free()


def _same(ids, cts, o_ids, o_cts):
    ids, cts = genie.as_uint32(ids), genie.as_uint32(cts)
    bad = np.nonzero((ids != o_ids).any(axis=1) | (cts != o_cts).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} rows differ, first {bad[0]}"


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("log2_slots", [2, 5])
def test_plain_path_overflows_exactly(case, persistent, log2_slots):
    inst, ix, off, items, o_ids, o_cts, _ = case
    print("overflow plain: slots", 1 << log2_slots, "persistent", persistent, flush=True)
    genie.genie_index_set_hash_slots(ix, log2_slots)
    genie.genie_index_set_scan_schedule(ix, persistent)
    try:
        ids, cts, ws = genie.genie_search_async(ix, off, items, inst.k,
                                                inst.queries.max_items())
        torch.cuda.synchronize()
    finally:
        genie.genie_index_set_hash_slots(ix, 0)
        genie.genie_index_set_scan_schedule(ix, 0)
    st = genie.workspace_stats(ws)
    assert st["status"] == 0, st
    assert st["ht_overflow_tiles"] > 0, st
    _same(ids, cts, o_ids, o_cts)


def test_default_table_does_not_overflow(case):
    inst, ix, off, items, o_ids, o_cts, _ = case
    ids, cts, ws = genie.genie_search_async(ix, off, items, inst.k, inst.queries.max_items())
    torch.cuda.synchronize()
    st = genie.workspace_stats(ws)
    assert st["ht_overflow_tiles"] == 0, st
    _same(ids, cts, o_ids, o_cts)


@pytest.mark.parametrize("persistent", [0, 1])
def test_gated_path_overflows_exactly(case, persistent):
    inst, ix, off, items, o_ids, o_cts, o_kth = case
    nq = inst.queries.n_queries
    # the exact k-th count for most queries, too high for every fifth (their
    # k-th count lies below the start, so they are answered again with AT = 1)
    pred = o_kth.astype(np.float32)
    pred[::5] += 3.0
    d_pred = torch.from_numpy(pred).cuda()
    print("overflow gated: persistent", persistent, flush=True)
    genie.genie_index_set_hash_slots(ix, 2)
    genie.genie_index_set_scan_schedule(ix, persistent)
    try:
        ids, cts, ws = genie.genie_search_gated_async(ix, off, items, inst.k,
                                                      inst.queries.max_items(), d_pred, 0.0)
        torch.cuda.synchronize()
    finally:
        genie.genie_index_set_hash_slots(ix, 0)
        genie.genie_index_set_scan_schedule(ix, 0)
    st = genie.workspace_stats(ws)
    assert st["status"] == 0, st
    assert st["ht_overflow_tiles"] > 0, st
    assert st["fallback_queries"] >= 1, st
    assert st["fallback_queries"] <= (nq + 4) // 5, st
    _same(ids, cts, o_ids, o_cts)


def test_rows_entry_point_overflows_exactly(case):
    inst, ix, off, items, o_ids, o_cts, _ = case
    nq = inst.queries.n_queries
    live = nq - 9
    rows = torch.tensor([live], dtype=torch.int32, device="cuda")
    ids = torch.full((nq, inst.k), -1, dtype=torch.int32, device="cuda")
    cts = torch.full_like(ids, -1)
    print("overflow rows: live", live, "of", nq, flush=True)
    genie.genie_index_set_hash_slots(ix, 3)
    try:
        ws = genie.alloc_workspace(ix, nq, inst.k)
        genie.genie_search_rows_async(ix, off, items, rows, inst.k, inst.queries.max_items(),
                                      ids, cts, ws)
        torch.cuda.synchronize()
    finally:
        genie.genie_index_set_hash_slots(ix, 0)
    _same(ids[:live], cts[:live], o_ids[:live], o_cts[:live])
    # rows past the live count are not written
    assert (genie.as_uint32(ids[live:]) == 0xFFFFFFFF).all()
