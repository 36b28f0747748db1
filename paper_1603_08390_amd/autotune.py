"""Autotuner for the scan kernel's launch shape.

For one index and a sample batch of its queries, every compiled shape
(threads per workgroup x posting dwords per thread and step) runs the search
a few times; the answers must be identical across shapes (they are a
function of the queries alone) and the fastest shape, by HIP-event time on
the search stream, is set on the index.  Results can be kept in a JSON cache
keyed by a workload name and the device name.
"""
from __future__ import annotations

import json
import os
from typing import Optional

from . import (SCAN_SHAPES, genie_index_set_scan_shape, genie_search_async, alloc_workspace)


def autotune(index, d_q_offsets, d_items, k: int, max_items: int, reps: int = 5,
             shapes=SCAN_SHAPES, cache_path: Optional[str] = None,
             key: Optional[str] = None) -> dict:
    import torch
    dev_name = torch.cuda.get_device_name()
    if cache_path and key and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        hit = cache.get(f"{key}|{dev_name}")
        if hit:
            genie_index_set_scan_shape(index, hit["threads"], hit["unroll"])
            return dict(hit, cached=True)
    nq = d_q_offsets.numel() - 1
    ws = alloc_workspace(index, nq, k)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    cts = torch.empty_like(ids)
    ref = None
    times = {}
    for (nt, u) in shapes:
        genie_index_set_scan_shape(index, nt, u)
        genie_search_async(index, d_q_offsets, d_items, k, max_items, ids, cts, ws)
        torch.cuda.synchronize()
        if ref is None:
            ref = (ids.clone(), cts.clone())
        elif not (torch.equal(ref[0], ids) and torch.equal(ref[1], cts)):
            raise RuntimeError(f"scan shape {nt}x{u} changed the answers")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            genie_search_async(index, d_q_offsets, d_items, k, max_items, ids, cts, ws)
        e1.record()
        torch.cuda.synchronize()
        times[f"{nt}x{u}"] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    nt, u = (int(x) for x in best.split("x"))
    genie_index_set_scan_shape(index, nt, u)
    out = {"threads": nt, "unroll": u, "ms": times, "cached": False}
    if cache_path and key:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[f"{key}|{dev_name}"] = {"threads": nt, "unroll": u, "ms": times}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return out
