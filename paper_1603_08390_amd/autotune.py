"""Autotuner for the index tiling and the scan kernel's launch shape.

`autotune`: for one index and a sample batch of its queries, every compiled
shape (threads per workgroup x posting dwords per thread and step) under
each schedule (one workgroup per pair, or persistent workgroups over a pair
queue) runs the search a few times; the answers must be identical across
them (they are a function of the queries alone) and the fastest, by
HIP-event time on the search stream, is set on the index.

`autotune_index`: builds the index with each tiling (tiles of 2^15 - 1 or
2^16 - 1 objects), tunes the shape on each, requires identical answers
across tilings, keeps the fastest index and frees the others.

Results can be kept in a JSON cache keyed by a workload name and the device
name.
"""
from __future__ import annotations

import json
import os
from typing import Optional

from . import (SCAN_SCHEDULES, SCAN_SHAPES, Index, alloc_workspace,
               genie_index_set_scan_schedule, genie_index_set_scan_shape, genie_search_async,
               genie_search_gated_async, queries_to_device)


def _label(nt, u, sched):
    return f"{nt}x{u}" + ("p" if sched else "")


def _apply(index, nt, u, sched):
    genie_index_set_scan_shape(index, nt, u)
    genie_index_set_scan_schedule(index, sched)


def autotune(index, d_q_offsets, d_items, k: int, max_items: int, reps: int = 5,
             shapes=SCAN_SHAPES, schedules=SCAN_SCHEDULES, cache_path: Optional[str] = None,
             key: Optional[str] = None, gate=None) -> dict:
    """Every (shape, schedule) on one index.  gate: None to tune the plain
    search, or (d_pred, delta) to tune the gated search with those per-query
    predictions.  Timings are keyed "threads x unroll", with a trailing "p"
    for the persistent schedule."""
    import torch
    hit = _cache_get(cache_path, key)
    if hit:
        _apply(index, hit["threads"], hit["unroll"], hit.get("persistent", 0))
        return dict(hit, cached=True)
    nq = d_q_offsets.numel() - 1
    ws = alloc_workspace(index, nq, k)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    cts = torch.empty_like(ids)

    def search():
        if gate is None:
            genie_search_async(index, d_q_offsets, d_items, k, max_items, ids, cts, ws)
        else:
            genie_search_gated_async(index, d_q_offsets, d_items, k, max_items, gate[0],
                                     gate[1], ids, cts, ws)

    ref = None
    times, configs = {}, {}
    for sched in schedules:
        for (nt, u) in shapes:
            _apply(index, nt, u, sched)
            search()
            torch.cuda.synchronize()
            if ref is None:
                ref = (ids.clone(), cts.clone())
            elif not (torch.equal(ref[0], ids) and torch.equal(ref[1], cts)):
                raise RuntimeError(f"scan shape {_label(nt, u, sched)} changed the answers")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                search()
            e1.record()
            torch.cuda.synchronize()
            times[_label(nt, u, sched)] = e0.elapsed_time(e1) / reps
            configs[_label(nt, u, sched)] = (nt, u, sched)
    best = min(times, key=times.get)
    nt, u, sched = configs[best]
    _apply(index, nt, u, sched)
    _cache_put(cache_path, key, {"threads": nt, "unroll": u, "persistent": sched, "ms": times})
    return {"threads": nt, "unroll": u, "persistent": sched, "ms": times, "cached": False}


def _cache_get(cache_path, key):
    import torch
    if not (cache_path and key and os.path.exists(cache_path)):
        return None
    with open(cache_path) as f:
        return json.load(f).get(f"{key}|{torch.cuda.get_device_name()}")


def _cache_put(cache_path, key, value):
    import torch
    if not (cache_path and key):
        return
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    cache[f"{key}|{torch.cuda.get_device_name()}"] = value
    with open(cache_path, "w") as f:
        json.dump(cache, f, indent=1)


def tune_tilings(indexes: dict, d_q_offsets, d_items, k: int, max_items: int,
                 shapes=SCAN_SHAPES, schedules=SCAN_SCHEDULES, reps: int = 3,
                 gate=None) -> dict:
    """Tune the scan shape on every index of {tile_log2: Index} (the same
    objects under different tilings) for one path (plain, or gated with
    gate = (d_pred, delta)); the answers must agree across tilings.  Every
    index is left at its own best shape.  Returns the best tiling and
    shape and all timings."""
    import torch
    nq = d_q_offsets.numel() - 1
    ref, best, report = None, None, {}
    for lg, ix in indexes.items():
        res = autotune(ix, d_q_offsets, d_items, k, max_items, reps=reps, shapes=shapes,
                       schedules=schedules, gate=gate)
        if gate is None:
            ids, cts, _ = genie_search_async(ix, d_q_offsets, d_items, k, max_items)
        else:
            ids, cts, _ = genie_search_gated_async(ix, d_q_offsets, d_items, k, max_items,
                                                   gate[0], gate[1])
        torch.cuda.synchronize()
        if ref is None:
            ref = (ids, cts)
        elif not (torch.equal(ref[0], ids) and torch.equal(ref[1], cts)):
            raise RuntimeError(f"tiling 2^{lg} - 1 changed the answers")
        ms = min(res["ms"].values())
        report[str(lg)] = res["ms"]
        if best is None or ms < best[1]:
            best = (lg, ms, res["threads"], res["unroll"], res["persistent"])
    lg, ms, nt, u, sched = best
    return {"tile_log2": lg, "threads": nt, "unroll": u, "persistent": sched, "ms": report,
            "queries": nq, "path": "plain" if gate is None else "gated"}


def autotune_index(values, n_buckets: int, q_offsets, items, k: int, max_items: int,
                   tilings=(16, 15), shapes=SCAN_SHAPES, schedules=SCAN_SCHEDULES, reps: int = 3,
                   cache_path: Optional[str] = None, key: Optional[str] = None):
    """Build the index with the fastest tiling and scan shape for the plain
    search of a sample batch (host q_offsets / items).  Returns (index,
    report)."""
    hit = _cache_get(cache_path, key)
    if hit:
        ix = Index(values, n_buckets, hit["tile_log2"])
        _apply(ix, hit["threads"], hit["unroll"], hit.get("persistent", 0))
        return ix, dict(hit, cached=True)
    off, it = queries_to_device(q_offsets, items)
    indexes = {lg: Index(values, n_buckets, lg) for lg in tilings}
    try:
        rep = tune_tilings(indexes, off, it, k, max_items, shapes=shapes, schedules=schedules,
                           reps=reps)
    except Exception:
        for ix in indexes.values():
            ix.free()
        raise
    for lg, ix in indexes.items():
        if lg != rep["tile_log2"]:
            ix.free()
    _cache_put(cache_path, key, {"tile_log2": rep["tile_log2"], "threads": rep["threads"],
                                 "unroll": rep["unroll"], "persistent": rep["persistent"]})
    return indexes[rep["tile_log2"]], dict(rep, cached=False)
