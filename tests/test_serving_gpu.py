"""Serving loop: each request's answer alone equals its answer in a mix of
requests of both shapes, several k, arriving while others run; admission
under a small device-memory budget queues requests instead of failing."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402
from paper_1603_08390_amd import serving  # noqa: E402

pytestmark = pytest.mark.gpu


def _residents():
    rel = workloads.relational(n=2 * 65535 + 321, d=16, V=64, nq=48)
    inp = workloads.ann(n=70_000, nq=40, m=64)
    P = torch.from_numpy(inp.points).cuda()
    lsh = {"a": torch.from_numpy(inp.a).cuda(), "b": torch.from_numpy(inp.b).cuda(),
           "rehash": torch.from_numpy(inp.rehash.view(np.int64)).cuda(), "w": inp.w,
           "log2_buckets": inp.log2_buckets}
    sig = genie.genie_lsh_signatures(P, lsh["a"], lsh["b"], inp.w, lsh["rehash"],
                                     inp.log2_buckets)
    torch.cuda.synchronize()
    ann_ix = genie.Index(genie.as_uint32(sig), 1 << inp.log2_buckets)
    res = {"rel": serving.Resident(genie.Index(rel.values, rel.V), rel.queries.max_items()),
           "ann": serving.Resident(ann_ix, inp.a.shape[0], lsh=lsh)}
    return rel, inp, res


def _requests(rel, inp, rng, rate):
    reqs = []
    t = serving.poisson_arrivals(rng, 88, rate)
    for i in range(88):
        k = int(rng.choice([10, 100, 1000]))
        if i % 2 == 0:
            q = int(rng.integers(0, rel.queries.n_queries))
            reqs.append(serving.Request(i, "rel", k, float(t[i]), items=rel.queries.items_of(q)))
        else:
            q = int(rng.integers(0, inp.queries.shape[0]))
            reqs.append(serving.Request(i, "ann", k, float(t[i]), point=inp.queries[q]))
    return reqs


def test_alone_equals_mix():
    rel, inp, res = _residents()
    reqs = _requests(rel, inp, np.random.default_rng(11), rate=4000.0)
    mixed = {r.rid: r for r in serving.Server(res, slots=3, max_batch=16).run(reqs)}
    assert len(mixed) == len(reqs)
    alone_srv = serving.Server(res, slots=1, max_batch=1)
    oidx = oracle.build_csr(rel.values, rel.V)
    for rq in reqs[:30]:
        one = serving.Request(rq.rid, rq.target, rq.k, 0.0, items=rq.items, point=rq.point)
        a = alone_srv.run([one])[0]
        m = mixed[rq.rid]
        assert np.array_equal(a.ids, m.ids) and np.array_equal(a.counts, m.counts), rq.rid
        if rq.target == "rel":
            q = workloads.Queries(np.array([0, len(rq.items)], np.uint64), rq.items)
            o_ids, o_cts, _, _ = oracle.search_idx(oidx, q, rq.k)
            assert np.array_equal(m.ids, o_ids[0]) and np.array_equal(m.counts, o_cts[0])
    s = serving.latency_summary(list(mixed.values()), max(r.done for r in mixed.values()))
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_admission_waits_for_memory():
    rel, inp, res = _residents()
    reqs = _requests(rel, inp, np.random.default_rng(5), rate=1e6)   # all at once
    ws = genie.genie_search_workspace_size(res["rel"].index, 2, 1000)
    srv = serving.Server(res, slots=4, max_batch=64, hbm_budget=3 * ws)
    out = srv.run(reqs)
    assert len(out) == len(reqs)
    assert srv.waited_for_memory > 0
    assert srv.in_use == 0


def test_graph_executor_equals_eager():
    """Groups replayed from HIP graphs recorded at the capacity (any group
    size through the device row count), with and without a gate model
    (untrained: its predictions send queries through the fallback), give
    the eager executor's answers bit for bit, and the oracle's."""
    from paper_1603_08390_amd import gate as gate_mod
    rel, inp, res = _residents()
    g = gate_mod.GateModel(seed=3)
    g.delta = 0.0
    res["rel"].gate = g
    rng = np.random.default_rng(21)
    reqs = _requests(rel, inp, rng, rate=3000.0)
    for use_gate in (False, True):
        eager = {r.rid: r for r in serving.Server(res, slots=2, max_batch=16,
                                                  use_gate=use_gate).run(reqs)}
        srv = serving.Server(res, slots=2, max_batch=16, use_gate=use_gate, graphs=True)
        graphed = {r.rid: r for r in srv.run(reqs)}
        assert isinstance(srv.ex, serving.GraphExecutor) and srv.ex.plans
        assert set(eager) == set(graphed) == {r.rid for r in reqs}
        for rid in eager:
            assert np.array_equal(eager[rid].ids, graphed[rid].ids), (use_gate, rid)
            assert np.array_equal(eager[rid].counts, graphed[rid].counts), (use_gate, rid)
    oidx = oracle.build_csr(rel.values, rel.V)
    for rq in reqs[:40]:
        if rq.target == "rel":
            q = workloads.Queries(np.array([0, len(rq.items)], np.uint64), rq.items)
            o_ids, o_cts, _, _ = oracle.search_idx(oidx, q, rq.k)
            assert np.array_equal(graphed[rq.rid].ids, o_ids[0])
            assert np.array_equal(graphed[rq.rid].counts, o_cts[0])
