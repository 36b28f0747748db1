"""CPU oracle for the learned initial gate -- TEST INFRASTRUCTURE ONLY.

Nothing in the paper corresponds to this part: the paper starts the
AuditThreshold at 1 (Section 3.3.1, Algorithm 1).  The gate model predicts a
query's k-th match count, which is the value AT - 1 reaches at the end of the
plain method (Theorem 3.1), so that AT can start near it.

Everything here is float64 numpy, written from the definitions:

* ``query_features`` -- the 64 input features of a query, from the posting
  counts of the keywords its items cover (no search needed).
* ``mlp_forward`` / ``pinball_loss`` / ``mlp_backward`` -- a 64-128-128-1
  network with ReLU hidden layers and a linear output, trained with the
  pinball (quantile) loss so that it errs low.
* ``adam_step`` -- the Adam update (Kingma and Ba) in float64.

Parameter layout (shared with the GPU kernels through the order of the flat
vector, not through code): W1 [128, 64], b1 [128], W2 [128, 128], b2 [128],
w3 [128], b3 [1], concatenated row-major.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

N_FEATURES = 64
H1 = 128
H2 = 128
SHAPES = (("W1", (H1, N_FEATURES)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
          ("w3", (H2,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation (float64)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((H1, N_FEATURES)) * math.sqrt(2.0 / N_FEATURES),
         "b1": np.zeros(H1),
         "W2": rng.standard_normal((H2, H1)) * math.sqrt(2.0 / H1),
         "b2": np.zeros(H2),
         "w3": rng.standard_normal(H2) * math.sqrt(1.0 / H2),
         "b3": np.zeros(1)}
    return flatten(p)


def to_bf16(theta: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  bfloat16 keeps the top 16 bits of a float32."""
    f = np.asarray(theta, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    r = (f + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return (r.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def bf16_bits(theta: np.ndarray) -> np.ndarray:
    """The uint16 bit patterns of to_bf16(theta)."""
    return (to_bf16(theta).astype(np.float32).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def mlp_forward(theta: np.ndarray, X: np.ndarray) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    """out = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 for every row of X."""
    p = unflatten(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["w3"] + p["b3"][0]
    return out, {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def pinball_loss(pred: np.ndarray, y: np.ndarray, tau: float) -> float:
    """Mean of tau * r for r = y - pred >= 0 and (tau - 1) * r otherwise."""
    r = np.asarray(y, dtype=np.float64) - np.asarray(pred, dtype=np.float64)
    return float(np.mean(np.where(r >= 0, tau * r, (tau - 1.0) * r)))


def pinball_grad(pred: np.ndarray, y: np.ndarray, tau: float) -> np.ndarray:
    """d(mean loss)/d(pred): -tau where y - pred >= 0, (1 - tau) elsewhere,
    divided by the batch size."""
    r = np.asarray(y, dtype=np.float64) - np.asarray(pred, dtype=np.float64)
    return np.where(r >= 0, -tau, 1.0 - tau) / float(len(r))


def mlp_backward(theta: np.ndarray, X: np.ndarray, y: np.ndarray, tau: float
                 ) -> Tuple[float, np.ndarray]:
    """Loss and its gradient with respect to the flat parameter vector."""
    p = unflatten(theta)
    out, c = mlp_forward(theta, X)
    loss = pinball_loss(out, y, tau)
    g = pinball_grad(out, y, tau)                 # [B]
    grads = {"w3": c["h2"].T @ g, "b3": np.array([g.sum()])}
    d2 = np.outer(g, p["w3"]) * (c["z2"] > 0)     # [B, H2]
    grads["W2"] = d2.T @ c["h1"]
    grads["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (c["z1"] > 0)           # [B, H1]
    grads["W1"] = d1.T @ c["X"]
    grads["b1"] = d1.sum(axis=0)
    return loss, flatten(grads)


def adam_step(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update; returns (theta, m, v).  step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------

def normal_quantile_upper(k: int, n: int) -> float:
    """z with P(Z > z) = k / n for a standard normal Z (k < n)."""
    from statistics import NormalDist
    q = min(max(k / float(n), 1e-12), 1 - 1e-12)
    return NormalDist().inv_cdf(1.0 - q)


def query_features(item_postings: np.ndarray, n: int, k: int) -> np.ndarray:
    """The 64 features of one query, from its items' posting counts.

    item_postings[i] = number of postings the index holds for the keywords of
    item i (its range on its dimension), so p_i = item_postings[i] / n is the
    fraction of objects that item i contains, and the match count of a
    random object has mean mu = sum p_i and variance sum p_i (1 - p_i).

      0  s / 512                         (s = number of items)
      1  mu / 64
      2  sigma / 8
      3  (mu + z sigma) / 64, z = upper k/n normal quantile
      4  max p_i
      5  sum p_i^2 / 64
      6  sum p_i^3 / 64
      7  z / 8
      8..23   histogram of the items with p_i > 0 by b = min(15, floor(-log2 p_i)),
              i.e. the largest b <= 15 with L_i * 2^b <= n (integers), / 64
      24..55  the 32 largest p_i, descending (0 when fewer items)
      56  number of items with p_i = 0, / 64
      57  number of items with p_i >= 0.25 (4 L_i >= n), / 64
      58..63  0
    """
    L = np.asarray(item_postings, dtype=np.float64)
    s = len(L)
    p = L / float(n)
    mu = float(p.sum())
    sigma = math.sqrt(float((p * (1.0 - p)).sum()))
    z = normal_quantile_upper(k, n)
    f = np.zeros(N_FEATURES, dtype=np.float64)
    f[0] = s / 512.0
    f[1] = mu / 64.0
    f[2] = sigma / 8.0
    f[3] = (mu + z * sigma) / 64.0
    f[4] = float(p.max()) if s else 0.0
    f[5] = float((p ** 2).sum()) / 64.0
    f[6] = float((p ** 3).sum()) / 64.0
    f[7] = z / 8.0
    for Li in np.asarray(item_postings, dtype=np.int64):
        if Li > 0:
            b = 0
            while b < 15 and int(Li) << (b + 1) <= n:
                b += 1
            f[8 + b] += 1.0 / 64.0
    top = np.sort(p)[::-1][:32]
    f[24:24 + len(top)] = top
    f[56] = float((p == 0).sum()) / 64.0
    f[57] = float((4 * np.asarray(item_postings, dtype=np.int64) >= n).sum()) / 64.0
    return f


def item_posting_counts(values: np.ndarray, items: np.ndarray, V: int) -> np.ndarray:
    """Postings covered by each item: objects whose value on the item's dim
    lies in [lo, min(hi, V-1)] (Definition 2.1 counted per item)."""
    values = np.asarray(values)
    out = np.zeros(len(items), dtype=np.int64)
    for i, (dim, lo, hi) in enumerate(np.asarray(items, dtype=np.int64).reshape(-1, 3)):
        col = values[:, dim]
        out[i] = int(((col >= lo) & (col <= min(hi, V - 1))).sum())
    return out
