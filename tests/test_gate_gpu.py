"""GPU parity of the learned gate against the float64 oracle, and exactness of
the gated search (identical to the plain search, fallbacks included)."""
import numpy as np
import pytest

import oracle
from oracle import gate_mlp as G
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402
from paper_1603_08390_amd import gate as gate_mod  # noqa: E402

pytestmark = pytest.mark.gpu

DISCRETE = list(range(8, 24)) + [56, 57]


def _feat_oracle(inst, k):
    rows = []
    for q in range(inst.queries.n_queries):
        L = G.item_posting_counts(inst.values, inst.queries.items_of(q), inst.V)
        rows.append(G.query_features(L, inst.n, k))
    return np.array(rows)


@pytest.mark.parametrize("which", ["relational", "uneven"])
def test_features_match_oracle(which):
    if which == "relational":
        inst = workloads.relational(n=150_000, d=16, V=64, nq=40)
    else:
        inst = workloads.uneven(n=140_000, d=16, V=64, nq=30, smin=1, smax=300)
    ix = genie.Index(inst.values, inst.V)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    f = genie.genie_gate_features_async(ix, off, items, 100)
    torch.cuda.synchronize()
    got = f.cpu().numpy().astype(np.float64)
    want = _feat_oracle(inst, 100)
    assert np.array_equal(got[:, DISCRETE], want[:, DISCRETE].astype(np.float32))
    cont = [c for c in range(64) if c not in DISCRETE]
    assert np.allclose(got[:, cont], want[:, cont], rtol=1e-6, atol=1e-7)
    ix.free()


def _rand_setup(n, seed):
    rng = np.random.default_rng(seed)
    theta = G.init_params(seed)
    X = rng.standard_normal((n, 64)).astype(np.float32)
    y = (rng.standard_normal(n) * 4 + 10).astype(np.float32)
    return theta, X, y


def test_forward_matches_oracle_bf16_and_f32():
    theta, X, _ = _rand_setup(300, 1)
    dX = torch.from_numpy(X).cuda()
    wb = torch.from_numpy(G.bf16_bits(theta).view(np.int16)).cuda()
    got = genie.genie_gate_forward_async(wb, dX).cpu().numpy()
    want, _ = G.mlp_forward(G.to_bf16(theta), X.astype(np.float64))
    assert np.allclose(got, want, rtol=1e-4, atol=1e-4 * np.abs(want).max())
    wf = torch.from_numpy(theta.astype(np.float32)).cuda()
    got32 = genie.genie_gate_forward_async(wf, dX).cpu().numpy()
    want32, _ = G.mlp_forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float64))
    assert np.allclose(got32, want32, rtol=1e-5, atol=1e-5 * np.abs(want32).max())
    # batch invariance: a row's prediction does not depend on its neighbours
    sub = genie.genie_gate_forward_async(wb, dX[37:181].contiguous()).cpu().numpy()
    assert np.array_equal(sub, got[37:181])


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_backward_matches_oracle(dtype):
    theta, X, y = _rand_setup(200, 2)
    dX, dy = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    if dtype == "bf16":
        w = torch.from_numpy(G.bf16_bits(theta).view(np.int16)).cuda()
        th = G.to_bf16(theta)
        rtol, atol_frac = 1e-2, 1e-3
    else:
        w = torch.from_numpy(theta.astype(np.float32)).cuda()
        th = theta.astype(np.float32).astype(np.float64)
        rtol, atol_frac = 1e-4, 1e-5
    grad, loss, _ = genie.genie_gate_backward_async(w, dX, dy, 0.1)
    torch.cuda.synchronize()
    want_loss, want = G.mlp_backward(th, X.astype(np.float64), y.astype(np.float64), 0.1)
    got = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - want_loss) <= 1e-4 * abs(want_loss) + 1e-6
    err = np.abs(got - want)
    assert np.all(err <= atol_frac * np.abs(want).max() + rtol * np.abs(want)), err.max()


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(3)
    master = rng.standard_normal(genie.GATE_PARAMS).astype(np.float32)
    grad = rng.standard_normal(genie.GATE_PARAMS).astype(np.float32)
    m0 = (rng.standard_normal(genie.GATE_PARAMS) * 0.1).astype(np.float32)
    v0 = np.abs(rng.standard_normal(genie.GATE_PARAMS) * 0.01).astype(np.float32)
    dm, dv = torch.from_numpy(m0.copy()).cuda(), torch.from_numpy(v0.copy()).cuda()
    dmaster = torch.from_numpy(master.copy()).cuda()
    dwb = torch.zeros(genie.GATE_PARAMS, dtype=torch.int16, device="cuda")
    genie.genie_gate_adam_async(dmaster, dwb, torch.from_numpy(grad).cuda(), dm, dv, 7, 1e-3)
    torch.cuda.synchronize()
    th, m, v = G.adam_step(master.astype(np.float64), grad.astype(np.float64),
                           m0.astype(np.float64), v0.astype(np.float64), 7, 1e-3)
    assert np.allclose(dmaster.cpu().numpy(), th, rtol=1e-5, atol=1e-6)
    assert np.allclose(dm.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
    got_bits = dwb.cpu().numpy().view(np.uint16)
    assert np.array_equal(got_bits, G.bf16_bits(dmaster.cpu().numpy().astype(np.float64)))


def _plain_and_gated(ix, queries, k, gate, delta):
    off, items = genie.queries_to_device(queries.q_offsets, queries.items)
    mi = max(1, queries.max_items())
    a_ids, a_cts, ws_a = genie.genie_search_async(ix, off, items, k, mi)
    g = torch.from_numpy(np.asarray(gate, dtype=np.float32)).cuda()
    b_ids, b_cts, ws_b = genie.genie_search_gated_async(ix, off, items, k, mi, g, delta)
    torch.cuda.synchronize()
    return (genie.as_uint32(a_ids), genie.as_uint32(a_cts), genie.workspace_stats(ws_a),
            genie.as_uint32(b_ids), genie.as_uint32(b_cts), genie.workspace_stats(ws_b))


@pytest.mark.parametrize("k,tile_log2", [(10, 16), (100, 16), (100, 15)])
def test_gated_search_is_exact(k, tile_log2):
    inst = workloads.relational(n=3 * 65535 + 99, d=12, V=48, nq=64, k=k)
    ix = genie.Index(inst.values, inst.V, tile_log2)
    oidx = oracle.build_csr(inst.values, inst.V)
    o_ids, o_cts, kth, _ = oracle.search_idx(oidx, inst.queries, k)
    rng = np.random.default_rng(k)
    cases = {
        "exact": kth.astype(np.float64) + 0.5,
        "too_high": kth.astype(np.float64) + 4.0,       # every query falls back
        "noisy": kth + rng.normal(0, 2.0, size=len(kth)),
        "zero": np.zeros(len(kth)),
        "nan": np.full(len(kth), np.nan),
        "huge": np.full(len(kth), 1e9),
    }
    for name, gate in cases.items():
        a_ids, a_cts, sa, b_ids, b_cts, sb = _plain_and_gated(ix, inst.queries, k, gate, 0.0)
        assert np.array_equal(a_ids, o_ids) and np.array_equal(a_cts, o_cts)
        assert np.array_equal(b_ids, o_ids), name
        assert np.array_equal(b_cts, o_cts), name
        assert sb["status"] == 0
        if name == "exact":
            assert sb["fallback_queries"] == 0
            assert sb["gate_passes"] < sa["gate_passes"]
        if name in ("too_high", "huge"):
            assert sb["fallback_queries"] == inst.queries.n_queries
    ix.free()


def test_trained_gate_cuts_gate_traffic_at_identical_results():
    """Train on one query set, apply to another: results identical to the
    plain method, far fewer increments through the gate, few fallbacks."""
    base = dict(n=2 * 65535 + 500, d=16, V=64, k=50)
    train = workloads.relational(nq=768, salt=100, **base)
    test = workloads.relational(nq=256, salt=0, **base)
    test.values = train.values   # same objects, different queries
    test.queries = workloads.queries_random_width(np.random.default_rng(7), train.values,
                                                  train.V, 256)
    ix = genie.Index(train.values, train.V)
    k = base["k"]

    def run(queries):
        off, items = genie.queries_to_device(queries.q_offsets, queries.items)
        ids, cts, ws = genie.genie_search_async(ix, off, items, k, queries.max_items())
        feats = genie.genie_gate_features_async(ix, off, items, k)
        torch.cuda.synchronize()
        return off, items, genie.as_uint32(ids), genie.as_uint32(cts), feats, \
            genie.workspace_stats(ws)

    _, _, _, tr_cts, tr_x, _ = run(train.queries)
    y = torch.from_numpy(tr_cts[:, k - 1].astype(np.float32)).cuda()
    model = gate_mod.GateModel(seed=1)
    losses = model.train(tr_x, y, epochs=40, batch=256, lr=2e-3, tau=0.1)
    assert losses[-1] < 0.5 * losses[0]
    pred_tr = model.predict(tr_x).cpu().numpy()
    model.calibrate(pred_tr, tr_cts[:, k - 1], target=0.02)

    off, items, ids, cts, x, st_plain = run(test.queries)
    pred = model.predict(x)
    g_ids, g_cts, ws = genie.genie_search_gated_async(ix, off, items, k, test.queries.max_items(),
                                                      pred, model.delta)
    torch.cuda.synchronize()
    st = genie.workspace_stats(ws)
    assert np.array_equal(genie.as_uint32(g_ids), ids)
    assert np.array_equal(genie.as_uint32(g_cts), cts)
    assert st["fallback_queries"] <= 0.1 * 256
    assert st["gate_passes"] < 0.6 * st_plain["gate_passes"], (st, st_plain)
    ix.free()
