"""Autotuner (every scan shape gives the same answers; the fastest is set)
and HIP-graph replay (every replay, with eager work in between, matches the
eager search on the same inputs)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402
from paper_1603_08390_amd import autotune, graph  # noqa: E402

pytestmark = pytest.mark.gpu


def test_autotune_shapes_agree_and_best_is_set(tmp_path):
    inst = workloads.relational(n=3 * 65535 + 17, d=16, V=64, nq=96)
    ix = genie.Index(inst.values, inst.V)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    cache = str(tmp_path / "tune.json")
    res = autotune.autotune(ix, off, items, 100, inst.queries.max_items(), reps=3,
                            cache_path=cache, key="relational-small")
    assert set(res["ms"]) == {f"{a}x{b}" + ("p" if sch else "") for sch in genie.SCAN_SCHEDULES
                              for a, b in genie.SCAN_SHAPES}
    best = f'{res["threads"]}x{res["unroll"]}' + ("p" if res["persistent"] else "")
    assert res["ms"][best] == min(res["ms"].values())
    assert ix.info.scan_shape == (res["threads"], res["unroll"])
    assert ix.info.scan_persistent == res["persistent"]
    again = autotune.autotune(ix, off, items, 100, inst.queries.max_items(), cache_path=cache,
                              key="relational-small")
    assert again["cached"] and again["threads"] == res["threads"]
    ids, cts, _ = genie.genie_search_async(ix, off, items, 100, inst.queries.max_items())
    o_ids, o_cts, _, _ = oracle.search_idx(oracle.build_csr(inst.values, inst.V),
                                           inst.queries, 100)
    assert np.array_equal(genie.as_uint32(ids), o_ids)
    assert np.array_equal(genie.as_uint32(cts), o_cts)
    ix.free()


def test_autotune_index_picks_a_tiling(tmp_path):
    inst = workloads.uneven(n=70_000, d=16, V=64, nq=32, smin=100, smax=300)
    cache = str(tmp_path / "tune.json")
    ix, rep = autotune.autotune_index(inst.values, inst.V, inst.queries.q_offsets,
                                      inst.queries.items, 50, inst.queries.max_items(), reps=2,
                                      cache_path=cache, key="uneven-small")
    assert set(rep["ms"]) == {"16", "15"}
    assert ix.info.tile_objects == (1 << rep["tile_log2"]) - 1
    assert ix.info.scan_shape == (rep["threads"], rep["unroll"])
    assert ix.info.scan_persistent == rep["persistent"]
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    ids, cts, _ = genie.genie_search_async(ix, off, items, 50, inst.queries.max_items())
    o_ids, o_cts, _, _ = oracle.search_idx(oracle.build_csr(inst.values, inst.V),
                                           inst.queries, 50)
    assert np.array_equal(genie.as_uint32(ids), o_ids)
    assert np.array_equal(genie.as_uint32(cts), o_cts)
    ix.free()
    ix2, rep2 = autotune.autotune_index(inst.values, inst.V, inst.queries.q_offsets,
                                        inst.queries.items, 50, inst.queries.max_items(),
                                        cache_path=cache, key="uneven-small")
    assert rep2["cached"] and ix2.info.tile_objects == (1 << rep["tile_log2"]) - 1
    ix2.free()


def test_graph_replays_match_eager():
    inst = workloads.relational(n=2 * 65535 + 5, d=12, V=48, nq=200)
    ix = genie.Index(inst.values, inst.V)
    nq_b = 40
    g = graph.GraphSearch(ix, nq_b, 50, 12, item_capacity=nq_b * 12)
    for rep in range(4):
        sub = inst.queries.subset(range(rep * nq_b, (rep + 1) * nq_b))
        ids, cts = g(sub.q_offsets, sub.items)
        got_ids, got_cts = genie.as_uint32(ids), genie.as_uint32(cts)
        # eager work between replays, and the eager answer for comparison
        off, items = genie.queries_to_device(sub.q_offsets, sub.items)
        e_ids, e_cts, _ = genie.genie_search_async(ix, off, items, 50, 12)
        torch.cuda.synchronize()
        assert np.array_equal(got_ids, genie.as_uint32(e_ids)), rep
        assert np.array_equal(got_cts, genie.as_uint32(e_cts)), rep
    ix.free()
