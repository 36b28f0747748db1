"""Pins of the float64 LSH oracle (Sections 4.1.2 and 4.2.3).

Hand-worked values fix the floor direction and the re-hash bit layout; the
closed form of the collision probability of Equation psi for p = 2 fixes the
projection arithmetic statistically; the re-hash is checked for range and a
pair-collision rate near 1/D (Theorem 4.1 uses omega = 1/D).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    with open(os.path.join(GOLD, "lsh_hand_values.json")) as f:
        return json.load(f)


def test_e2lsh_hand_values():
    g = _gold()["e2lsh"]
    h = oracle.e2lsh_f64(np.array(g["points"], dtype=np.float32),
                         np.array(g["a"], dtype=np.float32),
                         np.array(g["b"], dtype=np.float32), g["w"])
    assert h.tolist() == g["h"]


def test_rehash_hand_values():
    g = _gold()["rehash"]
    for c in g["cases"]:
        params = np.array([int(c["A"]), int(c["B"])], dtype=np.uint64)
        r = oracle.rehash(np.array([[c["h"]]], dtype=np.int64), params, g["log2_buckets"])
        assert int(r[0, 0]) == c["r"], c


def _phi(x):
    return 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))


def psi2(delta, w):
    """Equation psi for p = 2: phi is the half-normal density
    2/sqrt(2 pi) exp(-x^2/2); integrating t -> (1/delta) phi(t/delta)(1 - t/w)
    over [0, w] gives this closed form."""
    r = w / delta
    return (1.0 - 2.0 * _phi(-r)
            - (2.0 / (math.sqrt(2.0 * math.pi) * r)) * (1.0 - math.exp(-r * r / 2.0)))


def test_psi2_closed_form_matches_integral():
    from scipy import integrate
    w = 4.0
    for delta in (0.5, 1.0, 2.0, 4.0, 8.0):
        f = lambda t: (1.0 / delta) * (2.0 / math.sqrt(2 * math.pi)) * \
            math.exp(-(t / delta) ** 2 / 2.0) * (1.0 - t / w)
        val, _ = integrate.quad(f, 0.0, w)
        assert abs(val - psi2(delta, w)) < 1e-9
    # strictly decreasing in delta (Section 4.2.3)
    vals = [psi2(x, w) for x in np.linspace(0.1, 20, 50)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("delta", [0.5, 2.0, 6.0])
def test_e2lsh_collision_rate_matches_psi2(delta):
    """Empirical Pr[h(p) = h(q)] over random functions at ||p-q|| = delta."""
    rng = np.random.default_rng(1000 + int(delta * 10))
    dim, m, pairs, w = 32, 400, 200, 4.0
    a = rng.standard_normal((m, dim)).astype(np.float32)
    b = rng.uniform(0, w, size=m).astype(np.float32)
    p = rng.uniform(0, 10, size=(pairs, dim)).astype(np.float32)
    u = rng.standard_normal((pairs, dim))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q = (p + delta * u).astype(np.float32)
    # recompute the actual float32 distance so the pin is exact in delta
    hp = oracle.e2lsh_f64(p, a, b, w)
    hq = oracle.e2lsh_f64(q, a, b, w)
    coll = (hp == hq).mean()
    dd = np.linalg.norm(q.astype(np.float64) - p.astype(np.float64), axis=1)
    expect = np.mean([psi2(x, w) for x in dd])
    se = math.sqrt(expect * (1 - expect) / (m * pairs))
    assert abs(coll - expect) < 5 * se + 1e-3, (coll, expect)


def test_rehash_range_and_pair_collisions():
    rng = np.random.default_rng(4)
    m, L = 64, 13
    params = np.empty(2 * m, dtype=np.uint64)
    params[0::2] = rng.integers(0, 2 ** 63, size=m, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    params[1::2] = rng.integers(0, 2 ** 63, size=m, dtype=np.uint64)
    h1 = rng.integers(-5000, 5000, size=(4000, m))
    h2 = h1 + rng.integers(1, 5000, size=(4000, m))      # always a different signature
    r1 = oracle.rehash(h1, params, L)
    r2 = oracle.rehash(h2, params, L)
    assert r1.max() < 2 ** L and r2.max() < 2 ** L
    rate = (r1 == r2).mean()
    D = 2 ** L
    se = math.sqrt((1 / D) * (1 - 1 / D) / r1.size)
    assert abs(rate - 1.0 / D) < 6 * se + 2e-5, rate
    # equal signatures always collide
    assert np.array_equal(oracle.rehash(h1, params, L), r1)


def test_rehash_is_per_function():
    """Function i uses its own (A_i, B_i), stored interleaved: by hand,
    h = 1 with A_0 = 2^63+1 gives 4096 and with A_1 = 2^62+1 gives 2048."""
    params = np.array([2 ** 63 + 1, 0, 2 ** 62 + 1, 0], dtype=np.uint64)
    r = oracle.rehash(np.array([[1, 1]], dtype=np.int64), params, 13)
    assert r.tolist() == [[4096, 2048]]


def test_lsh_signatures_shape_and_determinism():
    inp = workloads.ann(n=2000, nq=50, m=37)
    s1 = oracle.lsh_signatures(inp.points, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    s2 = oracle.lsh_signatures(inp.points, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets,
                               chunk_rows=333)
    assert s1.shape == (2000, 37) and s1.dtype == np.uint32
    assert np.array_equal(s1, s2)
    assert s1.max() < 2 ** inp.log2_buckets


def test_near_points_share_more_buckets():
    """Theorem 4.1/4.2 in spirit: a query's own perturbed source point has a
    far larger match count than a random point."""
    inp = workloads.ann(n=3000, nq=40, m=64)
    sp = oracle.lsh_signatures(inp.points, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    sq = oracle.lsh_signatures(inp.queries, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    mc = (sp[None, :, :] == sq[:, None, :]).sum(axis=2)      # [nq, n]
    top = mc.max(axis=1)
    med = np.median(mc, axis=1)
    assert np.all(top > med + 10)


def test_theorem41_number_of_functions():
    """m = 2 ln(3/delta) / eps^2 at eps = delta = 0.06 is 2174 after rounding up."""
    m = 2 * math.log(3 / 0.06) / 0.06 ** 2
    assert math.ceil(m) == 2174
