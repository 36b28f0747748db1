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
               genie_search_gated_async, genie_search_rows_async, genie_search_workspace_size)


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

    def new_held_bytes(self, slot: int, group: List[Request]) -> int:
        """Device bytes that launching this group on this slot allocates and
        keeps for good (none: every buffer of an eager launch is released
        with the group)."""
        return 0

    def held_bytes(self) -> int:
        """Device bytes the executor keeps between groups."""
        return 0

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


class _Plan:
    """Device and pinned host buffers of one (slot, index, k) at the group
    capacity, and the HIP graph of its launches."""


class GraphExecutor(GpuExecutor):
    """Runs groups by replaying HIP graphs: one per (slot, index, k), recorded
    on first use at the group capacity, with the group's size passed as a
    device row count (genie_search_rows_async), so one graph serves every
    group size.  A launch is then the host-to-device copies of the group's
    inputs, one graph replay and the copy of the answers to pinned host
    memory, all on the slot's stream.  The graph holds kernels only (the
    library's status clear is a kernel, no memset node)."""

    def __init__(self, residents: Dict[str, Resident], slots: int, capacity: int,
                 use_gate: bool = True):
        super().__init__(residents, slots, use_gate)
        self.capacity = capacity
        self.plans = {}

    def _plan_bytes(self, target: str, k: int) -> int:
        """Device bytes of one plan at the group capacity (what _plan keeps)."""
        r, cap = self.res[target], self.capacity
        gated = self.use_gate and r.gate is not None
        if r.lsh is not None:
            m, dim = r.lsh["a"].shape[0], r.lsh["a"].shape[1]
            inputs = cap * dim * 4 + cap * m * 4 + cap * m * 12
        else:
            inputs = cap * max(1, r.max_items) * 12
        return (genie_search_workspace_size(r.index, cap, k) + 2 * cap * k * 4 + inputs +
                (cap + 1) * 8 + 4 + (cap * 64 * 4 + cap * 4 if gated else 0))

    def need_bytes(self, group: List[Request]) -> int:
        """A group runs in its plan's buffers: nothing beyond the plan."""
        return 0

    def new_held_bytes(self, slot: int, group: List[Request]) -> int:
        """The plan of (slot, index, k) is made on first use and kept."""
        key = (slot, group[0].target, group[0].k)
        return 0 if key in self.plans else self._plan_bytes(group[0].target, group[0].k)

    def held_bytes(self) -> int:
        return sum(P.bytes for P in self.plans.values())

    def release_held(self):
        """Drop every plan (only called while no group runs); they are made
        again on next use."""
        self.plans.clear()

    def _plan(self, slot: int, target: str, k: int) -> _Plan:
        key = (slot, target, k)
        if key in self.plans:
            return self.plans[key]
        torch, r, cap, dev = self.torch, self.res[target], self.capacity, "cuda"
        P = _Plan()
        P.rows = torch.zeros(1, dtype=torch.int32, device=dev)
        P.h_rows = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        if r.lsh is not None:
            m = r.lsh["a"].shape[0]
            dim = r.lsh["a"].shape[1]
            P.pts = torch.zeros((cap, dim), dtype=torch.float32, device=dev)
            P.h_pts = torch.zeros((cap, dim), dtype=torch.float32, pin_memory=True)
            P.sig = torch.zeros((cap, m), dtype=torch.int32, device=dev)
            P.off = torch.zeros(cap + 1, dtype=torch.int64, device=dev)
            P.items = torch.zeros((cap * m, 3), dtype=torch.int32, device=dev)
            P.max_items = m
        else:
            P.max_items = max(1, r.max_items)
            P.off = torch.zeros(cap + 1, dtype=torch.int64, device=dev)
            P.items = torch.zeros((cap * P.max_items, 3), dtype=torch.int32, device=dev)
            P.h_off = torch.zeros(cap + 1, dtype=torch.int64, pin_memory=True)
            P.h_items = torch.zeros((cap * P.max_items, 3), dtype=torch.int32, pin_memory=True)
        P.ids = torch.empty((cap, k), dtype=torch.int32, device=dev)
        P.cts = torch.empty((cap, k), dtype=torch.int32, device=dev)
        P.h_ids = torch.empty((cap, k), dtype=torch.int32, pin_memory=True)
        P.h_cts = torch.empty((cap, k), dtype=torch.int32, pin_memory=True)
        P.ws = alloc_workspace(r.index, cap, k, dev)
        gated = self.use_gate and r.gate is not None
        if gated:
            P.feats = torch.zeros((cap, 64), dtype=torch.float32, device=dev)
            P.pred = torch.zeros(cap, dtype=torch.float32, device=dev)

        def step():
            st = torch.cuda.current_stream()
            if r.lsh is not None:
                genie_lsh_signatures(P.pts, r.lsh["a"], r.lsh["b"], r.lsh["w"], r.lsh["rehash"],
                                     r.lsh["log2_buckets"], out=P.sig, stream=st)
                genie_lsh_items_async(P.sig, out=(P.off, P.items), stream=st)
            if gated:
                genie_gate_features_async(r.index, P.off, P.items, k, out=P.feats, stream=st)
                r.gate.predict(P.feats, out=P.pred, stream=st)
            genie_search_rows_async(r.index, P.off, P.items, P.rows, k, P.max_items, P.ids, P.cts,
                                    P.ws, d_gate=P.pred if gated else None,
                                    gate_delta=r.gate.delta if gated else 0.0, stream=st)

        st = self.streams[slot]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            step()                     # eager run: kernel attributes, allocator
        st.synchronize()
        P.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(P.graph, stream=st):
            step()
        st.synchronize()
        P.bytes = self._plan_bytes(target, k)
        self.plans[key] = P
        return P

    def launch(self, slot, group):
        torch = self.torch
        r = self.res[group[0].target]
        n, k = len(group), group[0].k
        if n > self.capacity:
            raise ValueError("group larger than the graph capacity")
        P = self._plan(slot, group[0].target, k)
        st = self.streams[slot]
        with torch.cuda.stream(st):
            if r.lsh is not None:
                P.h_pts[:n].numpy()[:] = np.stack([q.point for q in group])
                P.pts[:n].copy_(P.h_pts[:n], non_blocking=True)
            else:
                lens = [len(q.items) for q in group]
                o = P.h_off.numpy()
                o[0] = 0
                o[1:n + 1] = np.cumsum(lens)
                o[n + 1:] = o[n]               # rows past the group: empty queries
                if o[n]:
                    P.h_items.numpy()[:o[n]] = np.concatenate(
                        [q.items for q in group]).astype(np.uint32).reshape(-1, 3).view(np.int32)
                P.off.copy_(P.h_off, non_blocking=True)
                P.items[:max(1, o[n])].copy_(P.h_items[:max(1, o[n])], non_blocking=True)
            P.h_rows.numpy()[0] = n
            P.rows.copy_(P.h_rows, non_blocking=True)
            P.graph.replay()
            P.h_ids[:n].copy_(P.ids[:n], non_blocking=True)
            P.h_cts[:n].copy_(P.cts[:n], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"event": ev, "ids": P.h_ids[:n], "cts": P.h_cts[:n], "ws": P.ws}


class Server:
    """Continuous batching over `slots` execution slots.  The executor runs
    groups; this class decides when and what: arrival, grouping by (index,
    k), admission against the memory budget, completion."""

    def __init__(self, residents: Optional[Dict[str, Resident]] = None, slots: int = 4,
                 max_batch: int = 256, hbm_budget: Optional[int] = None, use_gate: bool = True,
                 executor=None, graphs: bool = False):
        if executor is None:
            executor = (GraphExecutor(residents, slots, max_batch, use_gate) if graphs else
                        GpuExecutor(residents, slots, use_gate))
        self.ex = executor
        self.n_slots = slots
        self.max_batch = max_batch
        self.budget = hbm_budget if hbm_budget is not None else int(self.ex.free_memory() * 0.5)
        self.in_use = 0
        self.waited_for_memory = 0
        self.released = 0
        self.groups = 0

    def run(self, requests: Sequence[Request], clock=time.perf_counter) -> List[Result]:
        reqs = sorted(requests, key=lambda q: q.arrival)
        # waiting requests, one arrival-ordered queue per (index, k); the
        # oldest head decides which group goes next
        queues: Dict[tuple, collections.deque] = {}
        n_waiting = 0
        results: List[Result] = []
        busy = [None] * self.n_slots     # (handle, group, bytes) per slot
        held_bytes = getattr(self.ex, "held_bytes", lambda: 0)
        new_held = getattr(self.ex, "new_held_bytes", lambda slot, group: 0)
        release = getattr(self.ex, "release_held", None)
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
            for _ in range(self.n_slots):          # admissions
                free = [j for j in range(self.n_slots) if busy[j] is None]
                if not free or not n_waiting:
                    break
                key = min((k for k, d in queues.items() if d), key=lambda k: queues[k][0].arrival)
                dq = queues[key]
                group = [dq.popleft() for _ in range(min(self.max_batch, len(dq)))]
                # a free slot that already holds what this kind of group needs
                i = min(free, key=lambda j: new_held(j, group))
                # device memory: what the group uses until it completes, plus
                # what launching it makes the executor keep for good (graph
                # plans), against the budget less what is in use or kept
                avail = self.budget - self.in_use - held_bytes()
                need = self.ex.need_bytes(group)
                hold = new_held(i, group)
                while need + hold > avail and len(group) > 1:
                    half = len(group) // 2
                    dq.extendleft(reversed(group[half:]))
                    group = group[:half]
                    need = self.ex.need_bytes(group)
                    hold = new_held(i, group)
                if need + hold > avail:
                    dq.extendleft(reversed(group))
                    if any(b is not None for b in busy):
                        self.waited_for_memory += 1
                        break                      # wait for a running group to finish
                    if held_bytes() > 0 and release is not None:
                        release()                  # nothing runs: drop what is kept, retry
                        self.released += 1
                        continue
                    raise MemoryError(f"one request needs {need + hold} bytes of device "
                                      f"memory; the budget is {self.budget}")
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
