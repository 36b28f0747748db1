"""Learned initial gate: a 64-128-128-1 MLP predicting a query's k-th match
count, trained and run by libgenie's kernels.

The paper's AuditThreshold starts at 1 (Algorithm 1); Theorem 3.1 says it
ends at the k-th count + 1.  Starting it near that value lets far fewer
increments through the gate.  Labels come from the plain method itself
(the k-th count of each training query); the pinball loss with a small
quantile makes the model err low, and a margin `delta` calibrated on the
training set keeps the share of queries that must be answered again (exact
fallback inside genie_search_gated_async) small.

This module only sequences calls into the library and moves parameters
between host files and device tensors.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from . import (GATE_FEATURES, GATE_PARAMS, genie_gate_adam_async, genie_gate_backward_async,
               genie_gate_features_async, genie_gate_forward_async)

# layout: W1 [128][64], b1 [128], W2 [128][128], b2 [128], w3 [128], b3
_SHAPES = ((128, 64), (128,), (128, 128), (128,), (128,), (1,))


def init_master(seed: int) -> np.ndarray:
    """He-style initial float32 master weights."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal((128, 64)) * math.sqrt(2.0 / 64), np.zeros(128),
             rng.standard_normal((128, 128)) * math.sqrt(2.0 / 128), np.zeros(128),
             rng.standard_normal(128) * math.sqrt(1.0 / 128), np.zeros(1)]
    flat = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert flat.size == GATE_PARAMS
    return flat


def bf16_bits_of(master: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 bit patterns (ties to even), as int16."""
    b = np.asarray(master, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16))
    return r.astype(np.uint16).view(np.int16)


class GateModel:
    """Device-resident gate model: float32 master weights, bf16 copy, Adam state."""

    def __init__(self, device="cuda", seed: int = 0, master: Optional[np.ndarray] = None):
        import torch
        self.device = device
        m = init_master(seed) if master is None else np.asarray(master, dtype=np.float32)
        self.master = torch.from_numpy(m.copy()).to(device)
        self.wbf = torch.from_numpy(bf16_bits_of(m)).to(device)
        self.m = torch.zeros(GATE_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros(GATE_PARAMS, dtype=torch.float32, device=device)
        self.step = 0
        self.delta = 0.0

    # -- inference -----------------------------------------------------------
    @staticmethod
    def features(index, d_q_offsets, d_items, k: int, stream=None):
        return genie_gate_features_async(index, d_q_offsets, d_items, k, stream=stream)

    def predict(self, d_x, out=None, stream=None):
        return genie_gate_forward_async(self.wbf, d_x, out=out, stream=stream)

    # -- training ------------------------------------------------------------
    def train(self, d_x, d_y, epochs: int = 30, batch: int = 512, lr: float = 1e-3,
              tau: float = 0.1, seed: int = 0) -> List[float]:
        """Adam on mini-batches of the pinball loss; returns the mean loss per
        epoch (computed by the backward kernel)."""
        import torch
        n = d_x.shape[0]
        rng = np.random.default_rng(seed)
        losses = []
        for _ in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).to(d_x.device)
            tot, cnt = 0.0, 0
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                xb = d_x.index_select(0, idx).contiguous()
                yb = d_y.index_select(0, idx).contiguous()
                grad, loss, _ = genie_gate_backward_async(self.wbf, xb, yb, tau)
                self.step += 1
                genie_gate_adam_async(self.master, self.wbf, grad, self.m, self.v, self.step, lr)
                tot += float(loss.item()) * len(idx)
                cnt += len(idx)
            losses.append(tot / max(cnt, 1))
        return losses

    def calibrate(self, pred: np.ndarray, kth: np.ndarray, target: float = 0.01) -> float:
        """Smallest margin delta (in steps of 0.25) such that at most `target`
        of the queries would start AT above their k-th count + 1 (and need
        the fallback): AT0 = floor(pred - delta), fallback iff kth < AT0 - 1."""
        pred = np.asarray(pred, dtype=np.float64)
        kth = np.asarray(kth, dtype=np.float64)
        for i in range(0, 400):
            d = 0.25 * i
            at0 = np.maximum(1.0, np.floor(pred - d))
            if np.mean(kth < at0 - 1) <= target:
                self.delta = d
                return d
        self.delta = 100.0
        return self.delta

    # -- checkpoint ----------------------------------------------------------
    def state(self) -> dict:
        return {"master": self.master.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": np.array([self.step]),
                "delta": np.array([self.delta])}

    def save(self, path: str):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str, device="cuda") -> "GateModel":
        import torch
        with np.load(path, allow_pickle=False) as z:
            g = cls(device=device, master=z["master"])
            g.m = torch.from_numpy(z["m"]).to(device)
            g.v = torch.from_numpy(z["v"]).to(device)
            g.step = int(z["step"][0])
            g.delta = float(z["delta"][0])
        return g
