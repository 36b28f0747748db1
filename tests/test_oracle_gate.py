"""Pins of the float64 gate-model oracle (the learned initial AT).

The network, loss and optimiser are not in the paper; they are pinned to
the mathematics: central finite differences for every gradient, hand-worked
forward values, special cases of the pinball loss, the known first Adam
step, bfloat16 rounding of chosen values, and hand-worked features.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import gate_mlp as G
import workloads


def test_parameter_count():
    assert G.N_PARAMS == 128 * 64 + 128 + 128 * 128 + 128 + 128 + 1


def test_forward_hand_values():
    p = {name: np.zeros(shape) for name, shape in G.SHAPES}
    p["W1"][0, 0] = 1.0
    p["W2"][0, 0] = 2.0
    p["w3"][0] = 3.0
    p["b3"][0] = 0.5
    theta = G.flatten(p)
    X = np.zeros((3, 64))
    X[0, 0] = 1.5     # 3 * relu(2 * relu(1.5)) + 0.5 = 9.5
    X[1, 0] = -1.0    # relus cut it: 0.5
    X[2, 0] = 0.25    # 3 * 0.5 + 0.5 = 2.0
    out, _ = G.mlp_forward(theta, X)
    assert out.tolist() == [9.5, 0.5, 2.0]


def test_pinball_special_cases():
    assert G.pinball_loss(np.array([0.0]), np.array([2.0]), 0.1) == pytest.approx(0.2)
    assert G.pinball_loss(np.array([0.0]), np.array([-2.0]), 0.1) == pytest.approx(1.8)
    y = np.array([1.0, -3.0, 2.5]); pred = np.array([0.0, 0.0, 0.0])
    assert G.pinball_loss(pred, y, 0.5) == pytest.approx(0.5 * np.mean(np.abs(y)))
    assert G.pinball_loss(y, y, 0.3) == 0.0


@pytest.mark.parametrize("tau", [0.1, 0.5])
def test_gradient_matches_central_differences(tau):
    rng = np.random.default_rng(5)
    theta = G.init_params(3)
    X = rng.standard_normal((16, 64))
    y = rng.standard_normal(16) * 3
    loss, g = G.mlp_backward(theta, X, y, tau)
    idx = rng.choice(G.N_PARAMS, size=60, replace=False)
    idx = np.concatenate([idx, [G.N_PARAMS - 1, G.N_PARAMS - 2, 0]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        num = (G.pinball_loss(G.mlp_forward(tp, X)[0], y, tau) -
               G.pinball_loss(G.mlp_forward(tm, X)[0], y, tau)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-5 * abs(num), (i, num, g[i])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3])
    r = G.to_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                     # halfway: ties to even
    assert r[2] == 1.0 + 2 ** -7           # above halfway: up
    assert r[3] == -2.5                    # exactly representable
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert G.bf16_bits(np.array([1.0]))[0] == 0x3F80


def test_adam_first_step_is_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = G.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-4)


def test_features_hand_values():
    f = G.query_features(np.array([50, 25, 0, 100]), n=100, k=10)
    p = np.array([0.5, 0.25, 0.0, 1.0])
    assert f[0] == 4 / 512
    assert f[1] == pytest.approx(1.75 / 64)
    assert f[2] == pytest.approx(math.sqrt(0.25 + 0.1875) / 8)
    z = G.normal_quantile_upper(10, 100)
    assert z == pytest.approx(1.2815515655, abs=1e-8)
    assert f[3] == pytest.approx((1.75 + z * math.sqrt(0.4375)) / 64)
    assert f[4] == 1.0
    assert f[5] == pytest.approx((p ** 2).sum() / 64)
    # bins: 100 -> 0, 50 -> 1, 25 -> 2; the empty item has none
    assert f[8:24].tolist() == [1 / 64, 1 / 64, 1 / 64] + [0.0] * 13
    assert f[24:28].tolist() == [1.0, 0.5, 0.25, 0.0]
    assert f[56] == 1 / 64 and f[57] == 3 / 64
    assert not f[58:].any()


def test_item_posting_counts_match_index():
    inst = workloads.relational(n=4000, d=6, V=20, nq=5)
    idx = oracle.build_csr(inst.values, inst.V)
    for q in range(5):
        items = inst.queries.items_of(q)
        got = G.item_posting_counts(inst.values, items, inst.V)
        for (dim, lo, hi), c in zip(items, got):
            want = sum(len(idx.postings(int(dim), v)) for v in range(int(lo), min(int(hi), 19) + 1))
            assert c == want
