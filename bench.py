"""Benchmark: match-count top-k search with c-PQ on one MI355X.

A step is one pass of the whole search path over one batch: every query of
the relational workload (1,000,000 objects x 32 dims, per-dim Zipf(1.1) over
256 buckets, 1,024 range queries of one item per dim, k = 100) goes through
the scan + count + c-PQ kernel and the per-query merge, with the index, the
queries, the outputs and the workspace already resident in HBM.  Two paths
are timed, K steps each: the plain c-PQ (AuditThreshold from 1), and the
learned gate (query features + MLP prediction + gated search with its exact
fallback), trained beforehand on a separate query set; their answers must be
identical.  `value` is the faster of the two.

Prints one JSON line.  Besides throughput it reports
  roofline      the scan kernel's algorithmic bytes per launch divided by its
                mean HIP-event duration on the launch stream, against the
                8 TB/s HBM peak; `traffic` holds the HBM bytes per launch
                measured by rocprofv3 counters when a committed counter summary
                for this exact kernel source is present (else null);
  atomic_roof   counter increments per second against the measured rate of
                conflict-free LDS atomics;
  cpu_baseline  the CPU oracle (plain C inverted-index scan, one thread) on a
                bounded sample of the same batch.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/sec at k=100, 1M objects, oracle-exact; learned-gate vs plain c-PQ"
HBM_PEAK_GBS = 8000.0
# Conflict-free LDS atomic add (with return), lane-consecutive addresses,
# measured on MI355X: 8.34e12/s over the chip (13.6 per CU per 2.4 GHz clock).
LDS_ATOMIC_PEAK = 8.34e12
PMC_SUMMARY = os.path.join(ROOT, "profiles", "scan_cpq_relational_pmc.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1603_08390_amd", "csrc", "search.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per scan launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel source."""
    try:
        with open(PMC_SUMMARY) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    if pmc.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return pmc.get("hbm_bytes_per_launch")


def cpu_baseline(inst, budget_s: float):
    import oracle
    idx = oracle.build_csr(inst.values, inst.V)
    nq = inst.queries.n_queries
    done, t0 = 0, time.perf_counter()
    while done < nq and time.perf_counter() - t0 < budget_s:
        q1 = min(nq, done + 64)
        oracle.search_idx(idx, inst.queries, inst.k, done, q1)
        done = q1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {nq} queries of the same batch, one thread, "
                      f"{dt:.1f} s (inverted-index scan + count array + selection, plain C)",
            "cpu": platform.processor() or platform.machine()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle time for the CPU baseline (0 disables)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true", help="skip the learned-gate path")
    ap.add_argument("--gate-train-queries", type=int, default=4096)
    ap.add_argument("--gate-epochs", type=int, default=30)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 3 times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1603_08390_amd as genie
    import workloads

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return
    inst = workloads.relational()
    nq, k = inst.queries.n_queries, inst.k
    ix = genie.Index(inst.values, inst.V)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    max_items = inst.queries.max_items()
    out_ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    out_cts = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    ws = genie.alloc_workspace(ix, nq, k)
    stream = torch.cuda.current_stream()

    def plain_step():
        genie.genie_search_async(ix, off, items, k, max_items, out_ids, out_cts, ws, stream)

    # learned gate: trained (outside any timed region) on a separate set of
    # queries over the same objects, labels = k-th counts of the plain method
    gate_ids = torch.empty_like(out_ids)
    gate_cts = torch.empty_like(out_cts)
    gws = genie.alloc_workspace(ix, nq, k)
    model = None
    if not args.no_gate:
        from paper_1603_08390_amd import gate as gate_mod
        tq = workloads.queries_random_width(np.random.default_rng(workloads.BASE_SEED + 102),
                                            inst.values, inst.V, args.gate_train_queries)
        toff, titems = genie.queries_to_device(tq.q_offsets, tq.items)
        t_ids, t_cts, _ = genie.genie_search_async(ix, toff, titems, k, tq.max_items())
        tx = genie.genie_gate_features_async(ix, toff, titems, k)
        ty = t_cts[:, k - 1].float().contiguous()
        model = gate_mod.GateModel(seed=1)
        model.train(tx, ty, epochs=args.gate_epochs, batch=256, lr=2e-3, tau=0.1)
        model.calibrate(model.predict(tx).cpu().numpy(), ty.cpu().numpy(), target=0.01)
        feats = torch.empty((nq, 64), dtype=torch.float32, device="cuda")
        pred = torch.empty(nq, dtype=torch.float32, device="cuda")

    def gated_step():
        genie.genie_gate_features_async(ix, off, items, k, out=feats, stream=stream)
        model.predict(feats, out=pred, stream=stream)
        genie.genie_search_gated_async(ix, off, items, k, max_items, pred, model.delta,
                                       gate_ids, gate_cts, gws, stream)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        genie.genie_kernel_timing_read(reset=True)   # drop the warmup launches
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # timed regions: exactly K steps of each path; the plain path's kernels
    # carry HIP event pairs on the launch stream (the roofline's durations)
    genie.genie_kernel_timing_enable(True)
    genie.genie_kernel_timing_read(reset=True)
    elapsed_plain = timed(plain_step)
    kt = genie.genie_kernel_timing_read(reset=True)
    genie.genie_kernel_timing_enable(False)
    stats = genie.workspace_stats(ws)
    if stats["status"] != 0:
        raise RuntimeError(f"device status {stats}")
    scanned = stats["postings_scanned"]
    elapsed_gate = timed(gated_step) if model is not None else None
    gstats = genie.workspace_stats(gws) if model is not None else None
    if model is not None:
        same = bool(torch.equal(gate_ids, out_ids) and torch.equal(gate_cts, out_cts))
        if not same:
            raise RuntimeError("gated and plain answers differ")

    scan_ms = kt["scan_ms"] / max(1, kt["scan_launches"])
    merge_ms = kt["merge_ms"] / max(1, kt["merge_launches"])

    qps_plain = nq * args.steps / elapsed_plain
    use_gate = model is not None and elapsed_gate < elapsed_plain
    elapsed = elapsed_gate if use_gate else elapsed_plain
    ms_per_step = elapsed * 1e3 / args.steps
    qps = nq * args.steps / elapsed

    # algorithmic bytes of one scan launch: postings (uint16, read once), the
    # items (12 B), two Position Map offsets per item per tile (8 B), and the
    # answer (8 B per result)
    s_total = int(inst.queries.q_offsets[-1])
    T = ix.info.n_tiles
    alg_bytes = 2 * scanned + 12 * s_total + 8 * s_total * T + 8 * k * nq
    achieved_gbs = alg_bytes / (scan_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "scan_cpq_kernel",
                "kernel_ms": round(scan_ms, 4), "merge_kernel_ms": round(merge_ms, 4),
                "alg_bytes_per_launch": alg_bytes}
    atomic_rate = scanned / (scan_ms * 1e-3)
    atomic_roof = {"achieved": atomic_rate, "peak": LDS_ATOMIC_PEAK, "unit": "increments/s",
                   "frac": round(atomic_rate / LDS_ATOMIC_PEAK, 4),
                   "postings_per_step": scanned}

    result = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "relational: 1,000,000 objects x 32 dims, per-dim Zipf(1.1) "
                               "over 256 buckets; 1,024 queries, one range item per dim, "
                               "width U{0..8}; k=100",
                   "n_objects": inst.n, "n_dims": inst.d, "n_buckets": inst.V,
                   "n_queries": nq, "k": k,
                   "path": "learned gate + c-PQ (exact fallback)" if use_gate else "plain c-PQ",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "atomic_roof": atomic_roof,
        "plain_cpq": {"value": round(qps_plain, 1),
                      "ms_per_step": round(elapsed_plain * 1e3 / args.steps, 4),
                      "gate_passes_per_step": stats["gate_passes"],
                      "ht_inserts_per_step": stats["ht_inserts"],
                      "ht_overflow_tiles": stats["ht_overflow_tiles"]},
        "learned_gate": None if model is None else {
            "value": round(nq * args.steps / elapsed_gate, 1),
            "ms_per_step": round(elapsed_gate * 1e3 / args.steps, 4),
            "speedup_vs_plain": round(elapsed_plain / elapsed_gate, 4),
            "identical_results": True,
            "gate_passes_per_step": gstats["gate_passes"],
            "fallback_queries_per_step": gstats["fallback_queries"],
            "delta": model.delta, "train_queries": args.gate_train_queries,
            "epochs": args.gate_epochs},
    }
    if not args.no_cpu_baseline and args.cpu_budget > 0:
        result["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget)
    else:
        result["cpu_baseline"] = None
    ix.free()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
