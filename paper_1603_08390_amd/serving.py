"""Continuous-batching request loop over resident indexes.

Requests (a relational query as items, or an ANN query as a point) arrive
over time.  The loop keeps a few execution slots, each a HIP stream with its
own device buffers; whenever a slot is free it takes the oldest waiting
request, groups it with the other waiting requests for the same index and k
(up to `max_batch`), and launches the group: for points, LSH signatures and
their exact-match items; then features and the gate prediction when a gate
model is set; then the search (plain or gated); then the copy of the answers
to pinned host memory.  Groups on different slots overlap on the device.  A
group is admitted only while the device memory it needs fits the budget
(free device memory at start-up, or a given number of bytes); otherwise it
waits until a running group finishes.

Every query's answer depends only on that query (the kernels never mix
queries), so a request gets the same answer alone and in any mix.  Latency is
measured from a request's arrival to the moment the loop sees its group's
completion event.

Orchestration only: every computation runs in libgenie's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import (Index, alloc_workspace, as_uint32, genie_gate_features_async,
               genie_lsh_items_async, genie_lsh_signatures, genie_search_async,
               genie_search_gated_async, genie_search_workspace_size)


@dataclasses.dataclass
class Resident:
    """One resident index and what its requests need."""
    index: Index
    max_items: int
    lsh: Optional[dict] = None          # {"a","b","rehash" device tensors, "w", "log2_buckets"}
    gate: Optional[object] = None       # gate.GateModel


@dataclasses.dataclass
class Request:
    rid: int
    target: str                          # name of a Resident
    k: int
    arrival: float                       # seconds from the start of the run
    items: Optional[np.ndarray] = None   # [s, 3] uint32 (relational)
    point: Optional[np.ndarray] = None   # [dim] float32 (ANN)


@dataclasses.dataclass
class Result:
    rid: int
    ids: np.ndarray
    counts: np.ndarray
    arrival: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class GpuExecutor:
    """Runs groups of requests on HIP streams through libgenie."""

    def __init__(self, residents: Dict[str, Resident], slots: int, use_gate: bool = True):
        import torch
        self.torch = torch
        self.res = residents
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.use_gate = use_gate

    def free_memory(self) -> int:
        return int(self.torch.cuda.mem_get_info()[0])

    def need_bytes(self, group: List[Request]) -> int:
        r = self.res[group[0].target]
        nq, k = len(group), group[0].k
        s_total = sum(len(q.items) if q.items is not None else
                      (r.lsh["a"].shape[0] if r.lsh else 0) for q in group)
        ws = genie_search_workspace_size(r.index, nq, k)
        return ws + 2 * nq * k * 4 + s_total * 12 + (nq + 1) * 8 + nq * 64 * 4 + 4096

    def launch(self, slot: int, group: List[Request]):
        torch = self.torch
        st = self.streams[slot]
        r = self.res[group[0].target]
        k, nq, dev = group[0].k, len(group), "cuda"
        keep = []
        with torch.cuda.stream(st):
            if r.lsh is not None:
                pts = np.stack([b.point for b in group]).astype(np.float32)
                d_pts = torch.from_numpy(pts).pin_memory().to(dev, non_blocking=True)
                sig = genie_lsh_signatures(d_pts, r.lsh["a"], r.lsh["b"], r.lsh["w"],
                                           r.lsh["rehash"], r.lsh["log2_buckets"], stream=st)
                off, items = genie_lsh_items_async(sig, stream=st)
                keep += [d_pts, sig]
                max_items = r.lsh["a"].shape[0]
            else:
                lens = [len(b.items) for b in group]
                o = np.zeros(nq + 1, dtype=np.uint64)
                o[1:] = np.cumsum(lens)
                it = (np.concatenate([b.items for b in group]).astype(np.uint32)
                      if o[-1] else np.zeros((1, 3), np.uint32))
                off = torch.from_numpy(o.view(np.int64)).pin_memory().to(dev, non_blocking=True)
                items = torch.from_numpy(it.reshape(-1, 3).view(np.int32)).pin_memory().to(
                    dev, non_blocking=True)
                max_items = max(1, max(lens))
            ws = alloc_workspace(r.index, nq, k, dev)
            ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
            cts = torch.empty((nq, k), dtype=torch.int32, device=dev)
            if self.use_gate and r.gate is not None:
                x = genie_gate_features_async(r.index, off, items, k, stream=st)
                pred = r.gate.predict(x, stream=st)
                genie_search_gated_async(r.index, off, items, k, max_items, pred, r.gate.delta,
                                         ids, cts, ws, st)
                keep += [x, pred]
            else:
                genie_search_async(r.index, off, items, k, max_items, ids, cts, ws, st)
            h_ids = torch.empty((nq, k), dtype=torch.int32, pin_memory=True)
            h_cts = torch.empty((nq, k), dtype=torch.int32, pin_memory=True)
            h_ids.copy_(ids, non_blocking=True)
            h_cts.copy_(cts, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        keep += [off, items, ids, cts]
        return {"event": ev, "ids": h_ids, "cts": h_cts, "ws": ws, "keep": keep}

    def done(self, handle) -> bool:
        return handle["event"].query()

    def fetch(self, handle):
        return handle["ids"].numpy().view(np.uint32), handle["cts"].numpy().view(np.uint32)


class Server:
    """Continuous batching over `slots` execution slots.  The executor runs
    groups; this class decides when and what: arrival, grouping by (index,
    k), admission against the memory budget, completion."""

    def __init__(self, residents: Optional[Dict[str, Resident]] = None, slots: int = 4,
                 max_batch: int = 256, hbm_budget: Optional[int] = None, use_gate: bool = True,
                 executor=None):
        self.ex = executor if executor is not None else GpuExecutor(residents, slots, use_gate)
        self.n_slots = slots
        self.max_batch = max_batch
        self.budget = hbm_budget if hbm_budget is not None else int(self.ex.free_memory() * 0.5)
        self.in_use = 0
        self.waited_for_memory = 0
        self.groups = 0

    def run(self, requests: Sequence[Request], clock=time.perf_counter) -> List[Result]:
        reqs = sorted(requests, key=lambda q: q.arrival)
        # waiting requests, one arrival-ordered queue per (index, k); the
        # oldest head decides which group goes next
        queues: Dict[tuple, collections.deque] = {}
        n_waiting = 0
        results: List[Result] = []
        busy = [None] * self.n_slots     # (handle, group, bytes) per slot
        nxt = 0
        t0 = clock()
        while nxt < len(reqs) or n_waiting or any(b is not None for b in busy):
            now = clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                q = reqs[nxt]
                queues.setdefault((q.target, q.k), collections.deque()).append(q)
                n_waiting += 1
                nxt += 1
            for i, b in enumerate(busy):           # completions
                if b is not None and self.ex.done(b[0]):
                    done = clock() - t0
                    ids, cts = self.ex.fetch(b[0])
                    for j, q in enumerate(b[1]):
                        results.append(Result(q.rid, ids[j].copy(), cts[j].copy(), q.arrival,
                                              done))
                    self.in_use -= b[2]
                    busy[i] = None
            for i in range(self.n_slots):          # admissions
                if busy[i] is not None or not n_waiting:
                    continue
                key = min((k for k, d in queues.items() if d), key=lambda k: queues[k][0].arrival)
                dq = queues[key]
                group = [dq.popleft() for _ in range(min(self.max_batch, len(dq)))]
                need = self.ex.need_bytes(group)
                while need > self.budget - self.in_use and len(group) > 1:
                    half = len(group) // 2
                    dq.extendleft(reversed(group[half:]))
                    group = group[:half]
                    need = self.ex.need_bytes(group)
                if need > self.budget - self.in_use:
                    dq.extendleft(reversed(group))
                    self.waited_for_memory += 1
                    break                          # wait for a running group to finish
                n_waiting -= len(group)
                self.in_use += need
                self.groups += 1
                busy[i] = (self.ex.launch(i, group), group, need)
            if nxt < len(reqs) and not n_waiting and all(b is None for b in busy):
                time.sleep(max(0.0, min(0.001, reqs[nxt].arrival - (clock() - t0))))
        return results


def latency_summary(results: Sequence[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    return {"requests": len(results), "qps": len(results) / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else 0.0,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else 0.0,
            "mean_ms": float(lat.mean()) if len(lat) else 0.0}


def poisson_arrivals(rng, n: int, rate: float) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
