"""Benchmark: match-count top-k search with c-PQ on one MI355X.

A step is one pass of the whole search path over one batch of queries, with
the index, the queries, the outputs and the workspace already resident in
HBM.  Each path first runs K eager steps, with the library's HIP event
pairs around its own kernel launches (the kernel durations of the roofline),
then its step is recorded once in a HIP graph and K replays are timed (the
throughput); every replay's answers equal the eager ones.  Two paths are timed, K steps each, on the same batch: the plain c-PQ
(AuditThreshold from 1), and the learned gate (query features + MLP
prediction + gated search with its exact fallback), trained beforehand on a
separate query set over the same objects; their answers must be identical.
`value` is the faster of the two.

Workloads (--workload):
  tiny        10,000 objects x 16 dims, values uniform in [0, 64), 100
              queries of one [v-2, v+2] item per dim, k = 10 (launch-bound).
  relational  (default) 1,000,000 objects x 32 dims, per-dim Zipf(1.1) over
              256 buckets, 1,024 range queries of one item per dim, k = 100.
  ann         tau-ANN: 1,000,000 float32 points in 128-d, 237 E2LSH functions
              re-hashed into 8,192 buckets, 4,096 perturbed query points,
              k = 100.  A step hashes the query points (LSH kernel), forms
              their exact-match items and searches; recall@100 and the
              approximation ratio against exact l2 are reported.
  uneven      10,000,000 objects x 64 dims, Zipf(1.1) over 1,024 buckets,
              16,384 queries of 4..512 items in one launch, k = 100; the
              index tiling and the scan shape are picked by the autotuner
              first.
  laplace     ANN in the Laplacian kernel space: the ann points through 237
              RBH functions (sigma = 32) re-hashed by MurmurHash3 into 8,192
              buckets; hashing in the step; recall against exact L1.
  sequence    sequence search under edit distance: 5,000,000 title-like
              strings, 1,024 queries of 40 bytes with 20 % replaced; a step
              decomposes the queries into ordered 3-grams, takes the top-32
              candidates by match count and verifies them (Algorithm 2,
              k = 1) with the top-k certificate; the certified fraction and
              the exact top-1 rate on the CPU baseline's sample are reported.
  multiload   8,000,000 relational objects whose index streams to the device
              in 4 parts per batch (multiple loadings), against one resident
              index of the same objects.
  serving     requests mixing the relational and the ANN shapes at k in
              {10, 100, 1000} through the continuous-batching loop: the
              saturated rate (all requests at once), then Poisson arrivals at
              0.3, 0.5, 0.7 and 0.9x the saturated plain rate (0.7 is the
              headline), with the learned gate off and on; p50/p99 latency and
              queries/s, and each (index, k) group's device time alone.

Prints one JSON line.  Besides throughput it reports
  roofline      the scan kernel's algorithmic bytes per launch divided by its
                mean HIP-event duration on the launch stream, against the
                8 TB/s HBM peak; `traffic` holds the HBM bytes per launch
                measured by rocprofv3 counters when a committed counter summary
                for this exact kernel source and workload is present (else
                null);
  atomic_roof   counter increments per second against the measured rate of
                conflict-free LDS atomics;
  cpu_baseline  the CPU oracle (plain C inverted-index scan) on the host's
                cores (up to 16 threads; the one-thread rate beside it) over a
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
METRICS = {
    "relational": METRIC,
    "tiny": "queries/sec at k=10, 10K objects x 16 dims (launch-bound); learned-gate vs plain c-PQ",
    "ann": "queries/sec at k=100, tau-ANN 1M points x 128-d, LSH hashing included; "
           "learned-gate vs plain c-PQ",
    "uneven": "queries/sec at k=100, 10M objects, 16,384 uneven queries in one launch; "
              "learned-gate vs plain c-PQ",
    "multiload": "queries/sec at k=100, 8M objects, index streamed in 4 parts per batch",
    "laplace": "queries/sec at k=100, Laplacian-kernel ANN via RBH, 1M points x 128-d, hashing "
               "included; learned-gate vs plain c-PQ",
    "serving": "queries/sec and p50/p99 latency of the request loop, relational + tau-ANN mix, "
               "k in {10,100,1000}; learned gate off and on",
    "sequence": "queries/sec, sequence search under edit distance, 5M strings, query length 40 "
                "with 20% modified, 3-grams, K=32 candidates, k=1; decomposition, verification "
                "and certificate included; learned-gate vs plain c-PQ",
}
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_1603_08390_amd", "csrc", "search.hip")


def log(*a):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def pmc_summary_path(workload: str, path: str = "plain") -> str:
    tag = "" if path == "plain" else "_" + path
    return os.path.join(ROOT, "profiles", f"scan_cpq_{workload}{tag}_pmc.json")


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str, path: str = "plain"):
    """HBM bytes per scan launch from the committed rocprofv3 counter summary
    of this workload and path, only if it was taken on the current kernel
    source."""
    try:
        with open(pmc_summary_path(workload, path)) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    if pmc.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return pmc.get("hbm_bytes_per_launch")


def measure_peaks(genie) -> dict:
    """Peak rates measured on this device in this run (library probes): LDS
    atomic adds with return at conflict-free and at random words, without
    return at random words; a streaming HBM read and copy of 2 GiB buffers
    (well past the 256 MB Infinity Cache)."""
    log("probing LDS atomic and HBM peaks")
    peaks = {"lds_atomic_conflict_free": genie.genie_probe_lds_atomics(0),
             "lds_atomic_random": genie.genie_probe_lds_atomics(1),
             "lds_atomic_random_no_return": genie.genie_probe_lds_atomics(2),
             "lds_atomic_one_bank_per_lane": genie.genie_probe_lds_atomics(3)}
    rd, cp = genie.genie_probe_hbm(2 << 30, 5)
    peaks.update(hbm_read_gbs=round(rd, 1), hbm_copy_gbs=round(cp, 1),
                 hbm_spec_gbs=HBM_PEAK_GBS,
                 source="genie_probe_lds_atomics (1024-thread workgroups, 64 KB LDS each, 8 "
                        "independent atomics per lane) and genie_probe_hbm, in this run")
    return peaks


def roofs(scanned, s_total, nq, k, n_tiles, kernel_ms, peaks, traffic):
    """Both roofs of one scan launch and the one that binds.

    HBM: the algorithmic bytes of the survey's count -- 4 B per posting
    (uint32 ids, read once), 12 B per item, 16 B of list offsets per item and
    8 B per result -- over the kernel's duration, against 8 TB/s; beside it
    the bytes this layout reads (2 B per posting, 12 B per item, 8 B of
    Position Map per item and tile, 8 B per result) and the HBM bytes the
    counters measured.  LDS atomics: one increment per posting, against the
    measured conflict-free rate of LDS atomic adds with return (lanes on
    consecutive words); beside it the fraction of the rate measured when
    each lane hits its own bank at scattered rows, which is what a scan's
    addresses look like (about half the conflict-free rate).  When the
    algorithmic bytes arrive faster than HBM can deliver them (the layout
    moves 2 B per posting and the caches serve part of them), HBM cannot be
    the bound in these bytes.  With a counter summary of this kernel
    source present, the roof with the larger fraction of the two measured
    rates binds -- the HBM bytes the counters saw, and the atomics -- and
    an HBM roof whose algorithmic bytes exceed HBM's rate reports the
    measured bytes as achieved; without one, HBM binds only when the
    algorithmic bytes fit under its peak and their fraction is the larger."""
    t = kernel_ms * 1e-3
    alg = 4 * scanned + 12 * s_total + 16 * s_total + 8 * k * nq
    layout = 2 * scanned + 12 * s_total + 8 * s_total * n_tiles + 8 * k * nq
    hbm_gbs = alg / t / 1e9
    hbm_frac = hbm_gbs / HBM_PEAK_GBS
    rate = scanned / t
    lds_peak = peaks["lds_atomic_conflict_free"]
    lds_frac = rate / lds_peak
    meas_frac = traffic / t / 1e9 / HBM_PEAK_GBS if traffic else None
    if meas_frac is not None:   # the counters say how much HBM actually moved
        hbm_binds = meas_frac >= lds_frac
    else:
        hbm_binds = hbm_frac <= 1.0 and hbm_frac >= lds_frac
    out = {"kernel": "scan_cpq_kernel", "kernel_ms": round(kernel_ms, 4)}
    if hbm_binds and hbm_frac <= 1.0:
        out.update(bound="hbm", achieved=round(hbm_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=round(hbm_frac, 4), achieved_bytes="algorithmic")
    elif hbm_binds:
        out.update(bound="hbm", achieved=round(traffic / t / 1e9, 1), peak=HBM_PEAK_GBS,
                   unit="GB/s", frac=round(meas_frac, 4),
                   achieved_bytes="measured HBM bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                  "calibrated): the algorithmic bytes exceed what HBM can "
                                  "deliver, the L2 and Infinity Cache serving part of them")
    else:
        out.update(bound="lds_atomic", achieved=round(rate / 1e9, 1),
                   peak=round(lds_peak / 1e9, 1), unit="G atomic adds/s",
                   frac=round(lds_frac, 4))
    out.update(traffic=traffic,
               hbm_alg_bytes_per_launch=alg, hbm_alg_gbs=round(hbm_gbs, 1),
               hbm_alg_frac=round(hbm_frac, 4),
               layout_bytes_per_launch=layout,
               hbm_measured_gbs=(round(traffic / t / 1e9, 1) if traffic else None),
               hbm_measured_frac=(round(traffic / t / 1e9 / HBM_PEAK_GBS, 4) if traffic else None),
               lds_atomic_rate=round(rate / 1e9, 1), lds_atomic_frac=round(lds_frac, 4),
               lds_atomic_frac_of_random=round(rate / peaks["lds_atomic_random"], 4),
               lds_atomic_frac_of_one_bank_per_lane=round(
                   rate / peaks["lds_atomic_one_bank_per_lane"], 4),
               postings_per_launch=scanned)
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_threads() -> int:
    """Threads for the oracle: the CPUs this process may run on, at most 16
    (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(values, V, queries, k, budget_s: float, chunk: int = 64):
    """The oracle's inverted-index search (plain C, one query after another
    per thread) on the host cores: half the budget on one thread, half on
    `threads` threads taking chunks of queries from a shared cursor (ctypes
    calls release the interpreter lock).  Queries are taken from the front of
    the batch, wrapping around, until the budget is spent.  The answers of
    every query the multi-threaded leg reached are kept (row -> (ids,
    counts)) so that the GPU's answers to the same rows can be checked
    against them."""
    import threading
    import oracle
    log("cpu baseline")
    idx = oracle.build_csr(values, V)
    nq = queries.n_queries
    answers = {}

    def run(threads, budget, keep):
        state = {"next": 0, "done": 0}
        lock = threading.Lock()
        t0 = time.perf_counter()

        def worker():
            while True:
                with lock:
                    if time.perf_counter() - t0 >= budget:
                        return
                    q0 = state["next"] % nq
                    q1 = min(nq, q0 + chunk)
                    state["next"] += q1 - q0
                ids, cts, _, _ = oracle.search_idx(idx, queries, k, q0, q1)
                with lock:
                    state["done"] += q1 - q0
                    if keep:
                        for r in range(q0, q1):
                            answers.setdefault(r, (ids[r - q0], cts[r - q0]))

        ws = [threading.Thread(target=worker) for _ in range(threads)]
        for w in ws:
            w.start()
        for w in ws:
            w.join()
        return state["done"], time.perf_counter() - t0

    threads = host_threads()
    d1, t1 = run(1, budget_s / 2, False)
    dn, tn = run(threads, budget_s / 2, True)
    return {"value": dn / tn, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "single_thread_value": d1 / t1,
            "sample": f"{dn} queries of the same batch ({nq} queries, taken in order, wrapping "
                      f"around) on {threads} threads in {tn:.1f} s, and {d1} on one thread in "
                      f"{t1:.1f} s (inverted-index scan + count array + selection, plain C)",
            "cpu": cpu_model(), "host_cpus": os.cpu_count()}, answers


def digest_check(workload, ids, cts):
    """The whole answer against the committed digest of the oracle's full
    answer for this workload (tests/golden/<workload>_oracle_digest.json,
    written by tests/golden/make_oracle_digests.py), when there is one."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_oracle_digest.json")
    try:
        with open(path) as f:
            ref = json.load(f)
    except (OSError, ValueError):
        return None
    ids = np.ascontiguousarray(np.asarray(ids).view(np.uint32))
    cts = np.ascontiguousarray(np.asarray(cts).view(np.uint32))
    if ids.shape != (ref["n_queries"], ref["k"]):
        return {"match": False, "reason": f"answer shape {ids.shape} is not the digest's"}

    def digest(a, b):
        h = hashlib.sha256()
        h.update(a.astype("<u4").tobytes())
        h.update(b.astype("<u4").tobytes())
        return h.hexdigest()

    B = ref["block_rows"]
    blocks = [digest(ids[b:b + B], cts[b:b + B]) for b in range(0, ids.shape[0], B)]
    bad = [i for i, (x, y) in enumerate(zip(blocks, ref["block_sha256"])) if x != y]
    return {"match": digest(ids, cts) == ref["sha256"], "rows": int(ids.shape[0]),
            "mismatched_blocks": bad, "block_rows": B,
            "reference": os.path.relpath(path, ROOT)}


def oracle_check(answers, ids, cts, nq):
    """The GPU's answers (the timed batch's last step) against the oracle's
    answers to the same rows, element by element."""
    ids = np.asarray(ids).view(np.uint32)
    cts = np.asarray(cts).view(np.uint32)
    rows = sorted(answers)
    bad = [r for r in rows
           if not (np.array_equal(ids[r], answers[r][0]) and np.array_equal(cts[r], answers[r][1]))]
    return {"rows_checked": len(rows), "rows_matched": len(rows) - len(bad), "of": nq,
            "first_mismatch": bad[0] if bad else None,
            "compared": "ids and counts of every checked row, bit for bit, against the CPU "
                        "oracle (inverted-index scan, Definition 2.1 counts, order count desc "
                        "then id asc); the gated and GEN-SPQ answers equal the plain ones"}


def train_gate(genie, torch, ix, sets, epochs: int, args=None):
    """Gate model trained on (features, k-th count of the plain method) pairs
    of the given (d_q_offsets, d_items, max_items, k) query sets; with
    --load-gate it is read from a file a run with --save-gate wrote (so that
    a profiler run holds no training launches)."""
    from paper_1603_08390_amd import gate as gate_mod
    if args is not None and getattr(args, "load_gate", None):
        log("gate model from", args.load_gate)
        return gate_mod.GateModel.load(args.load_gate)
    xs, ys = [], []
    for (toff, titems, tmax, k) in sets:
        _, t_cts, _ = genie.genie_search_async(ix, toff, titems, k, tmax)
        xs.append(genie.genie_gate_features_async(ix, toff, titems, k))
        ys.append(t_cts[:, k - 1].float())
    tx = torch.cat(xs).contiguous()
    ty = torch.cat(ys).contiguous()
    model = gate_mod.GateModel(seed=1)
    log("training the gate on", tx.shape[0], "queries")
    model.train(tx, ty, epochs=epochs, batch=256, lr=2e-3, tau=0.1)
    model.calibrate(model.predict(tx).cpu().numpy(), ty.cpu().numpy(), target=0.01)
    if args is not None and getattr(args, "save_gate", None):
        model.save(args.save_gate)
    return model


class SearchBench:
    """Times the plain and the gated path over one resident batch.

    `prep(stream)` returns the device (q_offsets, items) of the batch for
    this step: constant tensors for item queries, or the output of the LSH
    kernels for point queries (their time is then part of the step)."""

    def __init__(self, genie, torch, ix, nq, k, max_items, prep, workload, peaks):
        self.genie, self.torch, self.ix = genie, torch, ix
        self.workload, self.peaks = workload, peaks
        self.nq, self.k, self.max_items, self.prep = nq, k, max_items, prep
        self.stream = torch.cuda.current_stream()
        self.ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
        self.cts = torch.empty_like(self.ids)
        self.ws = genie.alloc_workspace(ix, nq, k)
        self.gids = torch.empty_like(self.ids)
        self.gcts = torch.empty_like(self.ids)
        self.feats = torch.empty((nq, 64), dtype=torch.float32, device="cuda")
        self.pred = torch.empty(nq, dtype=torch.float32, device="cuda")
        self.model = None
        # the gated path may run on the same objects under another tiling;
        # each path may have its own scan shape (set before its timed steps)
        self.plain_shape = None
        self.gate_shape = None
        self.spq = True
        # optional step after the search, on the same stream: post(st, ids, counts)
        self.post = None
        self.set_gate_index(ix)

    def set_gate_index(self, gix):
        self.gix = gix
        self.gws = self.genie.alloc_workspace(gix, self.nq, self.k)

    def plain_step(self):
        st = self.torch.cuda.current_stream()
        off, items = self.prep(st)
        self.genie.genie_search_async(self.ix, off, items, self.k, self.max_items, self.ids,
                                      self.cts, self.ws, st)
        if self.post:
            self.post(st, self.ids, self.cts)

    def gated_step(self):
        g, m = self.genie, self.model
        st = self.torch.cuda.current_stream()
        off, items = self.prep(st)
        g.genie_gate_features_async(self.gix, off, items, self.k, out=self.feats, stream=st)
        m.predict(self.feats, out=self.pred, stream=st)
        g.genie_search_gated_async(self.gix, off, items, self.k, self.max_items, self.pred,
                                   m.delta, self.gids, self.gcts, self.gws, st)
        if self.post:
            self.post(st, self.gids, self.gcts)

    def graphed(self, step):
        """Record one step in a HIP graph (after an eager run on the capture
        stream) and return its replay.  The library records kernels only
        (its status clear is a kernel, not a memset)."""
        torch = self.torch
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            step()
        torch.cuda.synchronize()
        self._graphs = getattr(self, "_graphs", []) + [graph]
        return graph.replay

    def timed(self, step, steps, warmup):
        """Warmup steps, then exactly `steps` steps between two device
        synchronisations; kernel event timings of the warmup are dropped."""
        torch, g = self.torch, self.genie
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        g.genie_kernel_timing_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def profile(self, path, steps, warmup):
        """Only one path's eager steps (profiler runs): the scan kernel's
        HIP-event mean duration, to set beside the profiler's."""
        g, torch = self.genie, self.torch
        step = self.plain_step if path == "plain" else self.gated_step
        ix = self.ix if path == "plain" else self.gix
        g.genie_kernel_timing_enable(True)
        g.genie_kernel_timing_read(reset=True)
        el = self.timed(step, steps, warmup)
        kt = g.genie_kernel_timing_read(reset=True)
        g.genie_kernel_timing_enable(False)
        st = g.workspace_stats(self.ws if path == "plain" else self.gws)
        return {"profile_path": path, "steps": steps, "warmup": warmup,
                "ms_per_step": round(el * 1e3 / steps, 4),
                "scan_kernel_ms": round(kt["scan_ms"] / max(1, kt["scan_launches"]), 4),
                "scan_launches": kt["scan_launches"],
                "merge_kernel_ms": round(kt["merge_ms"] / max(1, kt["merge_launches"]), 4),
                "postings_per_step": st["postings_scanned"] if path == "plain" else None,
                "stats": st, "tile_objects": ix.info.tile_objects,
                "scan_shape": "%dx%d" % tuple(ix.info.scan_shape),
                "schedule": schedule_name(ix, self.nq)}

    def run(self, steps, warmup, s_total, graph=False):
        """Each path: K eager steps with the library's kernel event pairs
        (the kernel durations), then, with graph=True, K replays of the step
        recorded in a HIP graph (the throughput); the replays must give the
        eager answers."""
        g, torch = self.genie, self.torch
        if self.plain_shape:
            g.genie_index_set_scan_shape(self.ix, *self.plain_shape[:2])
            g.genie_index_set_scan_schedule(self.ix, self.plain_shape[2])
        plain_shape = "%dx%d" % tuple(self.ix.info.scan_shape)
        plain_sched = schedule_name(self.ix, self.nq)
        g.genie_kernel_timing_enable(True)
        g.genie_kernel_timing_read(reset=True)
        el_plain = eager_plain = self.timed(self.plain_step, steps, warmup)
        kt = g.genie_kernel_timing_read(reset=True)
        log("plain path, eager:", round(eager_plain * 1e3 / steps, 3), "ms per step")
        g.genie_kernel_timing_enable(False)
        stats = g.workspace_stats(self.ws)
        if stats["status"] != 0:
            raise RuntimeError(f"device status {stats}")
        ref = (self.ids.clone(), self.cts.clone())
        if graph:
            replay = self.graphed(self.plain_step)
            self.ids.zero_()
            replay()
            torch.cuda.synchronize()
            if not (torch.equal(self.ids, ref[0]) and torch.equal(self.cts, ref[1])):
                raise RuntimeError("first graph replay and eager answers differ")
            el_plain = self.timed(replay, steps, warmup)
            if not (torch.equal(self.ids, ref[0]) and torch.equal(self.cts, ref[1])):
                raise RuntimeError("graph replay and eager answers differ")
        # GEN-SPQ ablation (Section 6.3): the same counters without the Gate
        # and the Hash Table; eager steps, against the eager plain c-PQ steps
        spq = None
        if self.spq:
            sids, scts = torch.empty_like(self.ids), torch.empty_like(self.cts)
            sws = g.alloc_workspace(self.ix, self.nq, self.k)

            def spq_step():
                st = torch.cuda.current_stream()
                off, items = self.prep(st)
                g.genie_search_spq_async(self.ix, off, items, self.k, self.max_items, sids, scts,
                                         sws, st)
                if self.post:
                    self.post(st, sids, scts)

            el_spq = self.timed(spq_step, steps, warmup)
            if not (torch.equal(sids, ref[0]) and torch.equal(scts, ref[1])):
                raise RuntimeError("GEN-SPQ and c-PQ answers differ")
            spq = {"value": round(self.nq * steps / el_spq, 1),
                   "ms_per_step": round(el_spq * 1e3 / steps, 4),
                   "cpq_speedup": round(el_spq / eager_plain, 4), "identical_results": True}
            log("GEN-SPQ, eager:", spq["ms_per_step"], "ms per step")
        el_gate, gstats, gkt, eager_gate = None, None, None, None
        if self.model is not None:
            if self.gate_shape:
                g.genie_index_set_scan_shape(self.gix, *self.gate_shape[:2])
                g.genie_index_set_scan_schedule(self.gix, self.gate_shape[2])
            g.genie_kernel_timing_enable(True)
            g.genie_kernel_timing_read(reset=True)
            el_gate = eager_gate = self.timed(self.gated_step, steps, warmup)
            gkt = g.genie_kernel_timing_read(reset=True)
            log("gated path, eager:", round(eager_gate * 1e3 / steps, 3), "ms per step")
            g.genie_kernel_timing_enable(False)
            gstats = g.workspace_stats(self.gws)
            if gstats["status"] != 0:
                raise RuntimeError(f"device status {gstats}")
            if not (torch.equal(self.gids, ref[0]) and torch.equal(self.gcts, ref[1])):
                raise RuntimeError("gated and plain answers differ")
            if graph:
                replay = self.graphed(self.gated_step)
                self.gids.zero_()
                replay()
                torch.cuda.synchronize()
                if not (torch.equal(self.gids, ref[0]) and torch.equal(self.gcts, ref[1])):
                    raise RuntimeError("first gated graph replay and plain answers differ")
                el_gate = self.timed(replay, steps, warmup)
                if not (torch.equal(self.gids, ref[0]) and torch.equal(self.gcts, ref[1])):
                    raise RuntimeError("gated graph replay and plain answers differ")

        nq, k = self.nq, self.k
        scan_ms = kt["scan_ms"] / max(1, kt["scan_launches"])
        merge_ms = kt["merge_ms"] / max(1, kt["merge_launches"])
        use_gate = el_gate is not None and el_gate < el_plain
        elapsed = el_gate if use_gate else el_plain
        scanned = stats["postings_scanned"]
        T = self.ix.info.n_tiles
        # the roofline belongs to the path whose throughput is `value`: its
        # main scan kernel (the gated path's fallback scan is a separate
        # launch, timed apart)
        if use_gate:
            kms = gkt["scan_ms"] / max(1, gkt["scan_launches"])
            roof_path, roof_T = "gated", self.gix.info.n_tiles
        else:
            kms, roof_path, roof_T = scan_ms, "plain", T
        roofline = roofs(scanned, s_total, nq, k, roof_T, kms, self.peaks,
                         measured_traffic(self.workload, roof_path))
        roofline.update(path=("learned gate + c-PQ" if use_gate else "plain c-PQ"),
                        merge_kernel_ms=round(merge_ms, 4))
        plain_roof = roofs(scanned, s_total, nq, k, T, scan_ms, self.peaks,
                           measured_traffic(self.workload, "plain"))
        rate = scanned / (scan_ms * 1e-3)
        atomic_roof = {"achieved": rate, "peak": self.peaks["lds_atomic_conflict_free"],
                       "unit": "increments/s", "path": "plain c-PQ",
                       "frac": round(rate / self.peaks["lds_atomic_conflict_free"], 4),
                       "postings_per_step": scanned}
        plain = {"value": round(nq * steps / el_plain, 1),
                 "ms_per_step": round(el_plain * 1e3 / steps, 4),
                 "eager_ms_per_step": round(eager_plain * 1e3 / steps, 4),
                 "scan_kernel_ms": round(scan_ms, 4),
                 "roofline": {key: plain_roof[key] for key in
                              ("bound", "achieved", "peak", "unit", "frac", "hbm_alg_frac",
                               "lds_atomic_frac")},
                 "gate_passes_per_step": stats["gate_passes"],
                 "ht_inserts_per_step": stats["ht_inserts"],
                 "ht_overflow_tiles": stats["ht_overflow_tiles"],
                 "tile_objects": self.ix.info.tile_objects,
                 "scan_shape": plain_shape, "schedule": plain_sched}
        learned = None
        if el_gate is not None:
            gms = gkt["scan_ms"] / max(1, gkt["scan_launches"])
            learned = {"value": round(nq * steps / el_gate, 1),
                       "ms_per_step": round(el_gate * 1e3 / steps, 4),
                       "eager_ms_per_step": round(eager_gate * 1e3 / steps, 4),
                       "speedup_vs_plain": round(el_plain / el_gate, 4),
                       "identical_results": True,
                       "gate_passes_per_step": gstats["gate_passes"],
                       "fallback_queries_per_step": gstats["fallback_queries"],
                       "scan_kernel_ms": round(gms, 4),
                       "fallback_scan_ms_per_step": round(gkt["fallback_ms"] / steps, 4),
                       "delta": self.model.delta,
                       "tile_objects": self.gix.info.tile_objects,
                       "scan_shape": "%dx%d" % tuple(self.gix.info.scan_shape),
                       "schedule": schedule_name(self.gix, self.nq)}
        return {"value": round(nq * steps / elapsed, 1),
                "ms_per_step": round(elapsed * 1e3 / steps, 4), "gen_spq": spq,
                "path": "learned gate + c-PQ (exact fallback)" if use_gate else "plain c-PQ",
                "launch": "HIP graph replay" if graph else "eager",
                "roofline": roofline, "atomic_roof": atomic_roof,
                "plain_cpq": plain, "learned_gate": learned}


def schedule_name(ix, nq):
    """The scan schedule a search of nq queries runs with on this index
    (schedule 2 is persistent from 1,024 (query, tile) pairs on)."""
    sched = ix.info.scan_persistent
    if sched == 2:
        sched = 1 if nq * ix.info.n_tiles >= 1024 else 0
    return "persistent" if sched == 1 else "grid"


def use_graph(args, workload):
    """HIP graph replay of the step (--graph on|off; auto: on)."""
    return args.graph in ("auto", "on")


def line(args, workload, res, config, dtype="u32"):
    out = {"metric": METRICS[workload], "value": res["value"], "unit": "queries/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": dict(config, path=res["path"], launch=res["launch"],
                          parallelism="single GPU",
                          step="the index, the queries, the answers and the workspace are "
                               "resident in HBM; host-device copies are outside the timed "
                               "step (the serving line's latencies include them)")}
    for key in ("roofline", "atomic_roof", "plain_cpq", "learned_gate", "gen_spq"):
        out[key] = res[key]
    out["peaks"] = args.peaks
    return out


def bench_item_queries(args, torch, genie, workloads, name, inst, train_queries, describe,
                       tune_sample=0, chunk=64):
    """Relational-style workloads: objects with one value per dim, queries of
    range items, all resident; `train_queries(rng)` draws the gate's
    training set over the same objects."""
    nq, k = inst.queries.n_queries, inst.k
    log(name, "generated:", inst.n, "objects,", nq, "queries")
    tune, indexes = None, {}
    if args.fixed:
        # a given tiling / shape / schedule for every path, no autotuning
        lg, nt, u, sched = args.fixed
        ix = genie.Index(inst.values, inst.V, lg)
        genie.genie_index_set_scan_shape(ix, nt, u)
        genie.genie_index_set_scan_schedule(ix, sched)
        tune_sample = 0
    elif tune_sample:
        # tiling and scan shape chosen by the autotuner on the batch's first
        # queries, for each path separately (index builds and tuning are
        # outside the timed regions)
        from paper_1603_08390_amd.autotune import tune_tilings
        sq = inst.queries.subset(range(min(nq, tune_sample)))
        soff, sitems = genie.queries_to_device(sq.q_offsets, sq.items)
        indexes = {lg: genie.Index(inst.values, inst.V, lg) for lg in (16, 15)}
        tune = {"plain": tune_tilings(indexes, soff, sitems, k, sq.max_items(), reps=2)}
        ix = indexes[tune["plain"]["tile_log2"]]
    else:
        ix = genie.Index(inst.values, inst.V)
    log("index ready:", ix.info)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    sb = SearchBench(genie, torch, ix, nq, k, inst.queries.max_items(), lambda st: (off, items),
                     name, args.peaks)
    if tune:
        sb.plain_shape = (tune["plain"]["threads"], tune["plain"]["unroll"],
                          tune["plain"]["persistent"])
    if not args.no_gate:
        tq = train_queries(np.random.default_rng(workloads.BASE_SEED + 100 + workloads.CONFIG_IDS[name]))
        n_train = tq.n_queries
        toff, titems = genie.queries_to_device(tq.q_offsets, tq.items)
        sb.model = train_gate(genie, torch, ix, [(toff, titems, tq.max_items(), k)],
                              args.gate_epochs, args)
        if tune:
            pred = sb.model.predict(genie.genie_gate_features_async(ix, soff, sitems, k))
            tune["gated"] = tune_tilings(indexes, soff, sitems, k, sq.max_items(), reps=2,
                                         gate=(pred, sb.model.delta))
            sb.set_gate_index(indexes[tune["gated"]["tile_log2"]])
            sb.gate_shape = (tune["gated"]["threads"], tune["gated"]["unroll"],
                             tune["gated"]["persistent"])
    for lg, other in indexes.items():
        if other is not sb.ix and other is not sb.gix:
            other.free()
    if args.profile_path:
        return sb.profile(args.profile_path, args.steps, args.warmup)
    res = sb.run(args.steps, args.warmup, int(inst.queries.q_offsets[-1]),
                 graph=use_graph(args, name))
    cfg = {"workload": describe, "n_objects": inst.n, "n_dims": inst.d, "n_buckets": inst.V,
           "n_queries": nq, "k": k}
    out = line(args, name, res, cfg)
    if tune is not None:
        # per path, per tiling (tile_log2), per scan shape
        out["autotune_ms"] = {path: t["ms"] for path, t in tune.items()}
    if out["learned_gate"]:
        out["learned_gate"].update(train_queries=n_train,
                                   epochs=args.gate_epochs)
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline and args.cpu_budget > 0:
        out["cpu_baseline"], answers = cpu_baseline(inst.values, inst.V, inst.queries, k,
                                                    args.cpu_budget, chunk=chunk)
        out["oracle_check"] = oracle_check(answers, genie.as_uint32(sb.ids),
                                           genie.as_uint32(sb.cts), nq)
    dig = digest_check(name, genie.as_uint32(sb.ids), genie.as_uint32(sb.cts))
    if dig is not None:
        out["oracle_digest"] = dig
    for used in {id(sb.ix): sb.ix, id(sb.gix): sb.gix}.values():
        used.free()
    return out


def bench_relational(args, torch, genie, workloads):
    inst = workloads.relational()
    return bench_item_queries(
        args, torch, genie, workloads, "relational", inst,
        lambda rng: workloads.queries_random_width(rng, inst.values, inst.V,
                                                   args.gate_train_queries),
        "relational: 1,000,000 objects x 32 dims, per-dim Zipf(1.1) over 256 buckets; 1,024 "
        "queries, one range item per dim, width U{0..8}; k=100")


def bench_tiny(args, torch, genie, workloads):
    inst = workloads.tiny()
    return bench_item_queries(
        args, torch, genie, workloads, "tiny", inst,
        lambda rng: workloads.queries_halfwidth(rng, inst.values, inst.V,
                                                args.gate_train_queries, 2),
        "tiny: 10,000 objects x 16 dims, values uniform in [0,64); 100 queries, one item "
        "[v-2, v+2] per dim; k=10")


def bench_uneven(args, torch, genie, workloads):
    inst = workloads.uneven()
    return bench_item_queries(
        args, torch, genie, workloads, "uneven", inst,
        lambda rng: workloads.queries_uneven(rng, inst.values, inst.V,
                                             args.gate_train_queries_uneven),
        "uneven: 10,000,000 objects x 64 dims, per-dim Zipf(1.1) over 1,024 buckets; 16,384 "
        "queries of U{4..512} range items in one launch; k=100", tune_sample=1024, chunk=1)


def lsh_device(torch, inp):
    return {"a": torch.from_numpy(inp.a).cuda(), "b": torch.from_numpy(inp.b).cuda(),
            "rehash": torch.from_numpy(inp.rehash.view(np.int64)).cuda(), "w": inp.w,
            "log2_buckets": inp.log2_buckets}


def ann_index(torch, genie, inp, lsh):
    """Index over the GPU LSH signatures of the points (built outside any
    timed region)."""
    sig = genie.genie_lsh_signatures(torch.from_numpy(inp.points).cuda(), lsh["a"], lsh["b"],
                                     lsh["w"], lsh["rehash"], lsh["log2_buckets"])
    torch.cuda.synchronize()
    sig_h = genie.as_uint32(sig)
    del sig
    return genie.Index(sig_h, 1 << inp.log2_buckets), sig_h


def exact_knn_gpu(torch, P, Q, k, chunk=256):
    """Exact l2 k nearest neighbours in float32 on the device (evaluation
    only: recall is a property of LSH, not of the search path)."""
    pn = (P * P).sum(1)
    ids, dist = [], []
    for i in range(0, Q.shape[0], chunk):
        q = Q[i:i + chunk]
        d2 = pn[None, :] - 2.0 * (q @ P.t()) + (q * q).sum(1)[:, None]
        v, j = torch.topk(d2, k, dim=1, largest=False)
        ids.append(j)
        dist.append(v.clamp_min(0).sqrt())
    return torch.cat(ids), torch.cat(dist)


def ann_quality(torch, P, Q, found, k):
    """recall@k and the approximation ratio (mean over queries of the mean
    ratio of the i-th found distance to the i-th true distance, both sorted;
    pairs with a zero true distance skipped)."""
    t_ids, t_dist = exact_knn_gpu(torch, P, Q, k)
    f = found.long()
    hit = (f[:, :, None] == t_ids[:, None, :]).any(2).float().mean().item()
    fd = ((P[f] - Q[:, None, :]) ** 2).sum(2).clamp_min(0).sqrt()
    fd, _ = torch.sort(fd, dim=1)
    ok = t_dist > 0
    r = torch.where(ok, fd / torch.where(ok, t_dist, torch.ones_like(t_dist)),
                    torch.zeros_like(fd))
    per_q = r.sum(1) / ok.sum(1).clamp_min(1)
    return hit, per_q[ok.any(1)].mean().item()


def bench_ann(args, torch, genie, workloads):
    inp = workloads.ann()
    log("ann generated")
    lsh = lsh_device(torch, inp)
    ix, sig_h = ann_index(torch, genie, inp, lsh)
    log("ann index ready:", ix.info)
    nq, m, k = inp.queries.shape[0], inp.a.shape[0], inp.k
    qpts = torch.from_numpy(inp.queries).cuda()
    qsig = torch.empty((nq, m), dtype=torch.int32, device="cuda")
    qoff = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    qitems = torch.empty((nq * m, 3), dtype=torch.int32, device="cuda")

    def prep(st):
        genie.genie_lsh_signatures(qpts, lsh["a"], lsh["b"], lsh["w"], lsh["rehash"],
                                   lsh["log2_buckets"], out=qsig, stream=st)
        genie.genie_lsh_items_async(qsig, out=(qoff, qitems), stream=st)
        return qoff, qitems

    sb = SearchBench(genie, torch, ix, nq, k, m, prep, "ann", args.peaks)
    if not args.no_gate:
        tq = workloads.ann_queries(np.random.default_rng(workloads.BASE_SEED + 103),
                                   inp.points, args.gate_train_queries)
        tsig = genie.genie_lsh_signatures(torch.from_numpy(tq).cuda(), lsh["a"], lsh["b"],
                                          lsh["w"], lsh["rehash"], lsh["log2_buckets"])
        toff, titems = genie.genie_lsh_items_async(tsig)
        sb.model = train_gate(genie, torch, ix, [(toff, titems, m, k)], args.gate_epochs, args)
    if args.profile_path:
        return sb.profile(args.profile_path, args.steps, args.warmup)
    res = sb.run(args.steps, args.warmup, nq * m, graph=use_graph(args, "ann"))
    P = torch.from_numpy(inp.points).cuda()
    rec, ratio = ann_quality(torch, P, qpts, sb.ids, k)
    out = line(args, "ann", res, {
        "workload": "tau-ANN: 1,000,000 float32 points x 128 (64-component Gaussian mixture, "
                    "clipped at 0); 237 E2LSH functions, w=4.0, re-hashed into 8,192 buckets; "
                    "4,096 perturbed query points; k=100",
        "n_objects": inp.points.shape[0], "n_functions": m, "n_buckets": 1 << inp.log2_buckets,
        "n_queries": nq, "k": k})
    out["quality"] = {"recall_at_100": round(rec, 4), "approximation_ratio": round(ratio, 4),
                      "queries": nq, "truth": "exact l2, float32 on the device"}
    if out["learned_gate"]:
        out["learned_gate"].update(train_queries=args.gate_train_queries,
                                   epochs=args.gate_epochs)
    if not args.no_cpu_baseline and args.cpu_budget > 0:
        qs = workloads.queries_exact(genie.as_uint32(qsig))
        cb, answers = cpu_baseline(sig_h, 1 << inp.log2_buckets, qs, k, args.cpu_budget)
        cb["sample"] += "; query signatures from the timed run, hashing not included"
        out["cpu_baseline"] = cb
        out["oracle_check"] = oracle_check(answers, genie.as_uint32(sb.ids),
                                           genie.as_uint32(sb.cts), nq)
        out["oracle_check"]["compared"] += ("; the oracle searches the device's signatures of "
                                            "the points and the queries (hashing is checked "
                                            "against the float64 oracle in the tests)")
    else:
        out["cpu_baseline"] = None
    ix.free()
    return out


def laplace_quality(torch, P, Q, found, k, sample=256):
    """recall@k against exact L1 neighbours (the Laplacian kernel is monotone
    in the L1 distance) and the L1 approximation ratio, on the first
    `sample` queries, in float32 on the device (evaluation only)."""
    Q, found = Q[:sample], found[:sample].long()
    rows = []
    for q0 in range(0, Q.shape[0], 16):
        q = Q[q0:q0 + 16, None, :]
        rows.append(torch.cat([(q - P[None, c:c + 32768]).abs().sum(-1)
                               for c in range(0, P.shape[0], 32768)], dim=1))
    d = torch.cat(rows, dim=0)
    t_dist, t_ids = torch.topk(d, k, dim=1, largest=False)
    hit = (found[:, :, None] == t_ids[:, None, :]).any(2).float().mean().item()
    fd, _ = torch.sort(torch.gather(d, 1, found), dim=1)
    ok = t_dist > 0
    r = torch.where(ok, fd / torch.where(ok, t_dist, torch.ones_like(t_dist)),
                    torch.zeros_like(fd))
    per_q = r.sum(1) / ok.sum(1).clamp_min(1)
    return hit, per_q[ok.any(1)].mean().item()


def bench_laplace(args, torch, genie, workloads):
    """ANN in the Laplacian kernel space (Section 4.1.3): the Gaussian-mixture
    points through 237 RBH functions re-hashed by MurmurHash3; a step hashes
    the query points (RBH kernel), forms their items and searches."""
    inp = workloads.laplace()
    log("laplace generated")
    g = torch.from_numpy(inp.g).cuda()
    u = torch.from_numpy(inp.u).cuda()
    seeds = torch.from_numpy(inp.seeds.view(np.int32)).cuda()
    sig = genie.genie_rbh_signatures(torch.from_numpy(inp.points).cuda(), g, u, seeds,
                                     inp.log2_buckets)
    torch.cuda.synchronize()
    sig_h = genie.as_uint32(sig)
    del sig
    ix = genie.Index(sig_h, 1 << inp.log2_buckets)
    log("laplace index ready:", ix.info)
    nq, m, k = inp.queries.shape[0], inp.g.shape[0], inp.k
    qpts = torch.from_numpy(inp.queries).cuda()
    qsig = torch.empty((nq, m), dtype=torch.int32, device="cuda")
    qoff = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    qitems = torch.empty((nq * m, 3), dtype=torch.int32, device="cuda")

    def prep(st):
        genie.genie_rbh_signatures(qpts, g, u, seeds, inp.log2_buckets, out=qsig, stream=st)
        genie.genie_lsh_items_async(qsig, out=(qoff, qitems), stream=st)
        return qoff, qitems

    sb = SearchBench(genie, torch, ix, nq, k, m, prep, "laplace", args.peaks)
    if not args.no_gate:
        tq = workloads.ann_queries(np.random.default_rng(workloads.BASE_SEED + 106),
                                   inp.points, args.gate_train_queries)
        tsig = genie.genie_rbh_signatures(torch.from_numpy(tq).cuda(), g, u, seeds,
                                          inp.log2_buckets)
        toff, titems = genie.genie_lsh_items_async(tsig)
        sb.model = train_gate(genie, torch, ix, [(toff, titems, m, k)], args.gate_epochs, args)
    if args.profile_path:
        return sb.profile(args.profile_path, args.steps, args.warmup)
    res = sb.run(args.steps, args.warmup, nq * m, graph=use_graph(args, "laplace"))
    P = torch.from_numpy(inp.points).cuda()
    rec, ratio = laplace_quality(torch, P, qpts, sb.ids, k)
    out = line(args, "laplace", res, {
        "workload": "Laplacian-kernel ANN: 1,000,000 float32 points x 128 (64-component "
                    "Gaussian mixture, clipped at 0); 237 RBH functions (sigma=32), "
                    "MurmurHash3 re-hash into 8,192 buckets; 4,096 perturbed query points; "
                    "k=100",
        "n_objects": inp.points.shape[0], "n_functions": m, "n_buckets": 1 << inp.log2_buckets,
        "n_queries": nq, "k": k})
    out["quality"] = {"recall_at_100": round(rec, 4), "l1_approximation_ratio": round(ratio, 4),
                      "queries": 256, "truth": "exact L1, float32 on the device"}
    if out["learned_gate"]:
        out["learned_gate"].update(train_queries=args.gate_train_queries,
                                   epochs=args.gate_epochs)
    if not args.no_cpu_baseline and args.cpu_budget > 0:
        qs = workloads.queries_exact(genie.as_uint32(qsig))
        cb, answers = cpu_baseline(sig_h, 1 << inp.log2_buckets, qs, k, args.cpu_budget)
        cb["sample"] += "; query signatures from the timed run, hashing not included"
        out["cpu_baseline"] = cb
        out["oracle_check"] = oracle_check(answers, genie.as_uint32(sb.ids),
                                           genie.as_uint32(sb.cts), nq)
        out["oracle_check"]["compared"] += ("; the oracle searches the device's signatures of "
                                            "the points and the queries (hashing is checked "
                                            "against the float64 oracle in the tests)")
    else:
        out["cpu_baseline"] = None
    ix.free()
    return out


def bench_multiload(args, torch, genie, workloads):
    """Multiple loadings (Section 3.4): 8,000,000 relational objects whose
    index is streamed to the device in four parts of 2,000,000 on every batch
    (pinned host memory -> two device slots, copies overlapped with the
    scans), against the same objects in one resident index."""
    inst = workloads.relational(n=8_000_000)
    nq, k = inst.queries.n_queries, inst.k
    log("multiload generated")
    part = 2_000_000
    parts = genie.PartsIndex(inst.values, inst.V, part)
    log("parts ready:", parts.info)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    mi = inst.queries.max_items()
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    cts = torch.empty_like(ids)
    ws = parts.workspace(nq, k)

    def step():
        genie.genie_parts_search_async(parts, off, items, k, mi, ids, cts, ws,
                                       torch.cuda.current_stream())

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        genie.genie_kernel_timing_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    genie.genie_kernel_timing_enable(True)
    el = timed(step)
    kt = genie.genie_kernel_timing_read(reset=True)
    genie.genie_kernel_timing_enable(False)
    stats = genie.workspace_stats(ws)
    if stats["status"] != 0:
        raise RuntimeError(f"device status {stats}")
    # the same objects in one resident index (the answers must agree)
    ix = genie.Index(inst.values, inst.V)
    rids = torch.empty_like(ids)
    rcts = torch.empty_like(ids)
    rws = genie.alloc_workspace(ix, nq, k)
    el_res = timed(lambda: genie.genie_search_async(ix, off, items, k, mi, rids, rcts, rws,
                                                    torch.cuda.current_stream()))
    if not (torch.equal(ids, rids) and torch.equal(cts, rcts)):
        raise RuntimeError("parts and resident answers differ")
    n_parts = parts.info["n_parts"]
    scan_ms = kt["scan_ms"] / max(1, kt["scan_launches"])
    scanned = stats["postings_scanned"]
    s_total = int(inst.queries.q_offsets[-1])
    T = parts.info["tiles_total"]
    step_ms = el * 1e3 / args.steps
    # one scan launch per part: a part's share of the postings and tiles
    roof = roofs(scanned // n_parts, s_total, nq, k, max(1, T // n_parts), scan_ms, args.peaks,
                 None)
    roof.update(scans_per_step=n_parts)
    h2d = parts.info["host_bytes"]
    out = {"metric": "queries/sec at k=100, 8M relational objects, index streamed in 4 parts "
                     "per batch (multiple loadings); oracle-exact",
           "value": round(nq * args.steps / el, 1), "unit": "queries/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic",
           "config": {"workload": "multiload: 8,000,000 objects x 32 dims, per-dim Zipf(1.1) "
                                  "over 256 buckets; 1,024 queries as relational; k=100; "
                                  "4 parts of 2,000,000 objects streamed every batch",
                      "n_objects": inst.n, "parts": n_parts, "part_objects": part,
                      "launch": "eager", "parallelism": "single GPU"},
           "roofline": roof, "peaks": args.peaks,
           "transfer": {"index_bytes_per_step": h2d,
                        "index_gbs_streamed": round(h2d / (step_ms * 1e-3) / 1e9, 2),
                        "scan_ms_per_step": round(scan_ms * n_parts, 4)},
           "resident_index": {"value": round(nq * args.steps / el_res, 1),
                              "ms_per_step": round(el_res * 1e3 / args.steps, 4),
                              "identical_results": True},
           "plain_cpq": {"postings_per_step": scanned}, "learned_gate": None}
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline and args.cpu_budget > 0:
        out["cpu_baseline"], answers = cpu_baseline(inst.values, inst.V, inst.queries, k,
                                                    args.cpu_budget)
        out["oracle_check"] = oracle_check(answers, genie.as_uint32(ids), genie.as_uint32(cts),
                                           nq)
    parts.free()
    ix.free()
    return out


def sequence_cpu_and_accuracy(inp, found_dist, budget_s: float):
    """The oracle's sequence search (match counts of every sequence, top-K,
    Algorithm 2) over the first queries of the batch until budget_s seconds,
    one thread; and, on those queries, whether the GPU's nearest distance is
    the true one over all sequences.  Only sequences whose count reaches
    |Q| - n + 1 - tau n (tau the GPU's distance) can be at distance tau or
    less (Theorem 5.1), so the exact minimum is taken over those."""
    from oracle import sequence as osq
    t0 = time.perf_counter()
    corpus = osq.SeqCorpus(inp.chars, inp.offsets, inp.gram)
    prep_s = time.perf_counter() - t0
    done, t_search, exact = 0, 0.0, 0
    while done < inp.nq and t_search < budget_s:
        q = inp.query(done)
        t1 = time.perf_counter()
        counts = corpus.match_counts(q)
        from oracle import topk_from_counts
        ids, cts = topk_from_counts(counts, inp.K)
        osq.verify(q, ids, cts, corpus.seq, inp.gram, inp.k)
        t_search += time.perf_counter() - t1
        tau = int(found_dist[done])
        theta = len(q) - inp.gram + 1 - tau * inp.gram
        cand = np.flatnonzero(counts >= theta)
        best = tau
        if cand.size:
            qb = np.frombuffer(q, np.uint8)
            d = osq.edit_distances(qb, np.array([0, len(q)], np.uint64),
                                   np.zeros(cand.size, np.uint64), corpus.chars, corpus.offsets,
                                   cand.astype(np.uint64))
            best = min(best, int(d.min()))
        exact += best == tau
        done += 1
    return ({"value": round(done / t_search, 3), "unit": "queries/s", "cores": 1,
             "kind": "oracle",
             "sample": f"the first {done} queries of the batch, one thread: match counts of all "
                       f"{inp.n} sequences (Lemma 5.1 over their windows), top-{inp.K}, "
                       f"Algorithm 2; window tables built once beforehand ({prep_s:.1f} s, "
                       "not timed)",
             "host": platform.processor() or platform.machine(), "nproc": os.cpu_count()},
            {"sample_queries": done, "top1_exact_fraction": round(exact / max(done, 1), 4)})


def bench_sequence(args, torch, genie, workloads):
    """Sequence search under edit distance (Section 5.1): 5,000,000
    title-like strings, 1,024 queries of 40 characters with 20 % of their
    characters replaced.  A step decomposes the queries into ordered 3-grams
    (device), takes the top-32 candidates by match count and verifies them
    (Algorithm 2, k = 1) with the certificate of Theorem 5.2.  The candidate
    search runs as plain c-PQ, with the learned gate (trained on other
    queries over the same strings), and as GEN-SPQ; all three give the same
    candidates, and every step includes decomposition and verification."""
    inp = workloads.sequence()
    log("sequence workload generated:", inp.n, "strings,", inp.chars.size, "bytes")
    sx = genie.SeqIndex(inp.chars, inp.offsets, inp.gram)
    log("sequence index ready:", sx.info)
    nq, K, k = inp.nq, inp.K, inp.k
    max_qlen = int(np.diff(inp.qoffsets).max())
    d_qc = torch.from_numpy(inp.qchars).cuda()
    d_qo = torch.from_numpy(inp.qoffsets.view(np.int64)).cuda()
    items = torch.empty((d_qc.numel(), 3), dtype=torch.int32, device="cuda")
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dist = torch.empty_like(ids)
    cert = torch.empty(nq, dtype=torch.int32, device="cuda")

    def prep(st):
        genie.genie_seq_decompose_async(sx, d_qc, d_qo, items, st)
        return d_qo, items

    def verify(st, c_ids, c_cts):
        genie.genie_seq_verify_async(sx, d_qc, d_qo, max_qlen, c_ids, c_cts, k, ids, dist, cert,
                                     st)

    ix = sx.match_index
    sb = SearchBench(genie, torch, ix, nq, K, max_qlen, prep, "sequence", args.peaks)
    sb.post = verify
    if not args.no_gate:
        rng = np.random.default_rng(workloads.BASE_SEED + 100 + workloads.CONFIG_IDS["sequence"])
        tq, to, _ = workloads.modified_queries(rng, inp.chars, inp.offsets,
                                               args.gate_train_queries, 40, 0.2)
        d_to = torch.from_numpy(to.view(np.int64)).cuda()
        titems = genie.genie_seq_decompose_async(sx, torch.from_numpy(tq).cuda(), d_to)
        sb.model = train_gate(genie, torch, ix, [(d_to, titems, 40, K)], args.gate_epochs)
    # items that name a keyword (the rest are empty and read nothing)
    prep(torch.cuda.current_stream())
    torch.cuda.synchronize()
    it = genie.as_uint32(items)
    s_total = int(np.count_nonzero(it[:, 1] <= it[:, 2]))
    res = sb.run(args.steps, args.warmup, s_total, graph=use_graph(args, "sequence"))
    # the answers of the last timed step (every path verifies the same candidates)
    torch.cuda.synchronize()
    dist_h, cert_h = genie.as_uint32(dist)[:, 0], genie.as_uint32(cert)
    out = line(args, "sequence", res, {
        "workload": "sequence: 5,000,000 title-like strings (4..14 words of a 30,000-word "
                    "Zipf(1.0) vocabulary, median 40 bytes); 1,024 queries of 40 bytes, 20% of "
                    "the bytes replaced; ordered 3-grams; K=32 candidates, k=1; decomposition "
                    "and verification in every step",
        "n_sequences": inp.n, "n_queries": nq, "K": K, "k": k, "gram": inp.gram})
    out["quality"] = {"certified_fraction": round(float(cert_h.mean()), 4),
                      "mean_top1_distance": round(float(dist_h.mean()), 3),
                      "max_top1_distance": int(dist_h.max())}
    out["index"] = sx.info
    if out["learned_gate"]:
        out["learned_gate"].update(train_queries=args.gate_train_queries,
                                   epochs=args.gate_epochs)
    if not args.no_cpu_baseline and args.cpu_budget > 0:
        cpu, acc = sequence_cpu_and_accuracy(inp, dist_h, args.cpu_budget)
        out["cpu_baseline"] = cpu
        out["quality"].update(acc)
    else:
        out["cpu_baseline"] = None
    sx.free()
    return out


def bench_serving(args, torch, genie, workloads):
    from paper_1603_08390_amd import serving
    rel = workloads.relational()
    inp = workloads.ann()
    lsh = lsh_device(torch, inp)
    ann_ix, _ = ann_index(torch, genie, inp, lsh)
    rel_ix = genie.Index(rel.values, rel.V)
    m = inp.a.shape[0]
    ks = (10, 100, 1000)
    gates = {"rel": None, "ann": None}
    if not args.no_gate:
        n_t = max(1, args.gate_train_queries // len(ks))
        tq = workloads.queries_random_width(np.random.default_rng(workloads.BASE_SEED + 105),
                                            rel.values, rel.V, n_t)
        toff, titems = genie.queries_to_device(tq.q_offsets, tq.items)
        gates["rel"] = train_gate(genie, torch, rel_ix,
                                  [(toff, titems, tq.max_items(), kk) for kk in ks],
                                  args.gate_epochs)
        tp = workloads.ann_queries(np.random.default_rng(workloads.BASE_SEED + 106),
                                   inp.points, n_t)
        tsig = genie.genie_lsh_signatures(torch.from_numpy(tp).cuda(), lsh["a"], lsh["b"],
                                          lsh["w"], lsh["rehash"], lsh["log2_buckets"])
        toff, titems = genie.genie_lsh_items_async(tsig)
        gates["ann"] = train_gate(genie, torch, ann_ix, [(toff, titems, m, kk) for kk in ks],
                                  args.gate_epochs)
    res = {"rel": serving.Resident(rel_ix, rel.queries.max_items(), gate=gates["rel"]),
           "ann": serving.Resident(ann_ix, m, lsh=lsh, gate=gates["ann"])}

    # one group of each (index, k) kind run alone, plain and gated: device
    # time of the group and the gated search's fallback queries
    groups = []
    rng = np.random.default_rng(workloads.BASE_SEED + 109)
    for target in ("rel", "ann"):
        for kk_ in ks:
            g = []
            for i in range(args.max_batch):
                if target == "rel":
                    q = int(rng.integers(0, rel.queries.n_queries))
                    g.append(serving.Request(i, "rel", kk_, 0.0, items=rel.queries.items_of(q)))
                else:
                    q = int(rng.integers(0, inp.queries.shape[0]))
                    g.append(serving.Request(i, "ann", kk_, 0.0, point=inp.queries[q]))
            row = {"target": target, "k": kk_, "requests": len(g)}
            log("serving group alone:", target, "k =", kk_)
            for use_gate in ((False, True) if not args.no_gate else (False,)):
                ex = serving.GpuExecutor(res, 1, use_gate)
                for _ in range(2):
                    ex.launch(0, g)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                reps = 5
                for _ in range(reps):
                    h = ex.launch(0, g)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps * 1e3
                st = genie.workspace_stats(h["ws"])
                row["gated_ms" if use_gate else "plain_ms"] = round(dt, 3)
                if use_gate:
                    row["fallback_queries"] = st["fallback_queries"]
            groups.append(row)

    rng = np.random.default_rng(workloads.BASE_SEED + 107)
    n_req = args.requests
    kind = rng.integers(0, 2, size=n_req)
    kk = rng.choice(ks, size=n_req)
    qrow = rng.integers(0, 1 << 30, size=n_req)

    def requests(arrivals):
        out = []
        for i in range(n_req):
            if kind[i] == 0:
                q = int(qrow[i] % rel.queries.n_queries)
                out.append(serving.Request(i, "rel", int(kk[i]), float(arrivals[i]),
                                           items=rel.queries.items_of(q)))
            else:
                q = int(qrow[i] % inp.queries.shape[0])
                out.append(serving.Request(i, "ann", int(kk[i]), float(arrivals[i]),
                                           point=inp.queries[q]))
        return out

    executors = {}

    def run(arrivals, use_gate, graphs=None):
        import gc
        graphs = args.serving_graphs if graphs is None else graphs
        key = (use_gate, graphs)
        if key not in executors:   # graphs are recorded once per executor
            executors[key] = (serving.GraphExecutor(res, args.slots, args.max_batch, use_gate)
                              if graphs else serving.GpuExecutor(res, args.slots, use_gate))
        srv = serving.Server(res, slots=args.slots, max_batch=args.max_batch,
                             executor=executors[key])
        batch = requests(arrivals)
        gc.collect()
        gc.disable()
        try:
            done = srv.run(batch)
        finally:
            gc.enable()
        wall = max(r.done for r in done)   # the loop's own clock: start -> last completion
        log("serving run:", "gate" if use_gate else "plain", "graphs" if graphs else "eager",
            len(batch), "requests,", srv.groups, "groups,", round(wall, 2), "s")
        s = serving.latency_summary(done, wall)
        s.update(groups=srv.groups, waited_for_memory=srv.waited_for_memory)
        return {r.rid: r for r in done}, {key: (round(v, 3) if isinstance(v, float) else v)
                                          for key, v in s.items()}

    zero = np.zeros(n_req)
    run(zero, False)                     # warm-up passes, not reported
    if not args.no_gate:
        run(zero, True)
    torch.cuda.synchronize()
    sat_plain_res, sat_plain = run(zero, False)
    sat_gate = None
    if not args.no_gate:
        sat_gate_res, sat_gate = run(zero, True)
        for rid, r in sat_plain_res.items():
            g = sat_gate_res[rid]
            if not (np.array_equal(r.ids, g.ids) and np.array_equal(r.counts, g.counts)):
                raise RuntimeError(f"request {rid}: gated and plain answers differ")
    # Poisson arrivals at fractions of the saturated plain rate, the same
    # arrival times for the plain and the gated run of each load
    loads = [float(x) for x in args.loads.split(",")]
    sweep = []
    for i, frac in enumerate(loads):
        rate_i = frac * sat_plain["qps"]
        arr = serving.poisson_arrivals(np.random.default_rng(workloads.BASE_SEED + 108 + i),
                                       n_req, rate_i)
        _, pp = run(arr, False)
        pg = run(arr, True)[1] if not args.no_gate else None
        sweep.append({"load": frac, "offered_qps": round(rate_i, 1), "plain": pp,
                      "learned_gate": pg})
    head = min(sweep, key=lambda r: abs(r["load"] - 0.7))
    rate, pois_plain, pois_gate = head["offered_qps"], head["plain"], head["learned_gate"]
    # the other executor at saturation and at the headline load, same arrivals
    other = not args.serving_graphs
    arr = serving.poisson_arrivals(
        np.random.default_rng(workloads.BASE_SEED + 108 + sweep.index(head)), n_req,
        head["offered_qps"])
    run(zero, False, other)
    compare = {"executor": "graph" if other else "eager",
               "saturated_plain": run(zero, False, other)[1],
               "poisson_plain": run(arr, False, other)[1]}
    if not args.no_gate:
        run(zero, True, other)
        compare["saturated_gate"] = run(zero, True, other)[1]
        compare["poisson_gate"] = run(arr, True, other)[1]
    best = pois_gate if pois_gate and pois_gate["qps"] > pois_plain["qps"] else pois_plain
    ms = n_req / best["qps"] * 1e3 if best["qps"] > 0 else 0.0   # the whole request stream
    out = {"metric": METRICS["serving"], "value": best["qps"], "unit": "queries/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic",
           "config": {"workload": "serving: relational (1M x 32, Zipf(1.1) over 256 buckets) "
                                  "and tau-ANN (1M x 128, 237 LSH functions) requests, 50/50, "
                                  f"k uniform in {{10,100,1000}}; Poisson arrivals at "
                                  f"{head['load']}x the saturated plain rate",
                      "requests": n_req, "slots": args.slots, "max_batch": args.max_batch,
                      "offered_qps": rate, "parallelism": "single GPU"},
           "saturated": {"plain": sat_plain, "learned_gate": sat_gate,
                         "identical_results": sat_gate is not None},
           "poisson": {"plain": pois_plain, "learned_gate": pois_gate},
           "load_sweep": sweep,
           "executor": "graph" if args.serving_graphs else "eager",
           "other_executor": compare,
           "groups": groups,
           "cpu_baseline": None}
    rel_ix.free()
    ann_ix.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 50; 3 for the uneven workload)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 5; 1 for the uneven workload)")
    ap.add_argument("--workload", choices=sorted(METRICS), default=None,
                    help="one workload alone; by default the relational headline with the "
                         "--nested workloads reported inside its line")
    ap.add_argument("--nested", default="tiny,ann,uneven,serving",
                    help="default run only: workloads reported under 'configs' in the "
                         "headline line, each with its own roofline and CPU baseline "
                         "('none' for the headline alone)")
    ap.add_argument("--time-budget", type=float, default=470.0,
                    help="default run only: a nested workload is skipped (and said so) when "
                         "its expected duration no longer fits this many seconds")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle time for the CPU baseline (0 disables)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true", help="skip the learned-gate path")
    ap.add_argument("--graph", choices=("auto", "on", "off"), default="auto",
                    help="time HIP graph replays of the step (auto: on); kernel durations "
                         "always come from an eager pass of the same steps")
    ap.add_argument("--gate-train-queries", type=int, default=4096)
    ap.add_argument("--gate-train-queries-uneven", type=int, default=16384,
                    help="queries the gate is trained on for the uneven workload")
    ap.add_argument("--gate-epochs", type=int, default=30)
    ap.add_argument("--fixed", default=None, metavar="L,T,U,P",
                    help="item workloads: tiles of 2^L-1 objects, T threads x U dwords, "
                         "schedule P (0 grid, 1 persistent) for every path instead of the "
                         "default or autotuned configuration (e.g. for profiler runs)")
    ap.add_argument("--requests", type=int, default=100000, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=4, help="serving: execution slots")
    ap.add_argument("--max-batch", type=int, default=256, help="serving: requests per group")
    ap.add_argument("--serving-executor", choices=("graph", "eager"), default="graph",
                    help="serving: replay per-(slot, index, k) HIP graphs, or launch eagerly")
    ap.add_argument("--loads", default="0.3,0.5,0.7,0.9",
                    help="serving: offered loads as fractions of the saturated plain rate")
    ap.add_argument("--profile-path", choices=("plain", "gated"), default=None,
                    help="profiler runs (item and ANN workloads): only this path's eager "
                         "steps; no graph, ablation, CPU baseline or nested workloads")
    ap.add_argument("--save-gate", default=None, metavar="PATH",
                    help="write the trained gate model here")
    ap.add_argument("--load-gate", default=None, metavar="PATH",
                    help="read the gate model from here instead of training it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 3 times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    args.serving_graphs = args.serving_executor == "graph"
    if args.fixed:
        args.fixed = tuple(int(x) for x in args.fixed.split(","))
        if len(args.fixed) != 4:
            ap.error("--fixed takes L,T,U,P")
    steps_given, warmup_given = args.steps, args.warmup
    set_steps(args, args.workload or "relational", steps_given, warmup_given)

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
    t_start = time.perf_counter()
    if args.profile_path:
        args.nested = "none"
        args.peaks = None
        out = {"relational": bench_relational, "tiny": bench_tiny, "ann": bench_ann,
               "uneven": bench_uneven, "laplace": bench_laplace}[args.workload or "relational"](
                   args, torch, genie, workloads)
        print(json.dumps(out), flush=True)
        return
    args.peaks = measure_peaks(genie)
    fns = {"relational": bench_relational, "tiny": bench_tiny, "ann": bench_ann,
           "uneven": bench_uneven, "serving": bench_serving,
           "multiload": bench_multiload, "laplace": bench_laplace,
           "sequence": bench_sequence}
    out = fns[args.workload or "relational"](args, torch, genie, workloads)
    if args.workload is None:
        out["configs"] = {}
        for name in [x for x in args.nested.split(",") if x and x != "none"]:
            left = args.time_budget - (time.perf_counter() - t_start)
            if NESTED_EXPECTED_S[name] > left:
                out["configs"][name] = {"skipped": f"expected {NESTED_EXPECTED_S[name]} s; "
                                                   f"{left:.0f} s of the time budget left"}
                log("skipping", name, "(time budget)")
                continue
            sub = argparse.Namespace(**vars(args))
            set_steps(sub, name, steps_given, warmup_given, nested=True)
            sub.cpu_budget = min(args.cpu_budget, NESTED_CPU_BUDGET_S)
            log("nested workload:", name)
            t0 = time.perf_counter()
            try:
                res = fns[name](sub, torch, genie, workloads)
            except Exception as e:   # reported in the line; the run's exit status says so
                res = {"error": f"{type(e).__name__}: {e}"}
            res["wall_s"] = round(time.perf_counter() - t0, 1)
            out["configs"][name] = res
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    out["wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)
    if not exact(out):
        log("answers differ from the oracle, or a nested workload failed")
        sys.exit(3)


# Expected duration of each nested workload on one MI355X, including input
# generation, index builds, tuning, gate training and the CPU baseline.
NESTED_EXPECTED_S = {"tiny": 30, "ann": 90, "uneven": 200, "serving": 150, "relational": 40,
                     "laplace": 90, "sequence": 120, "multiload": 90}
NESTED_CPU_BUDGET_S = 10.0


def set_steps(args, workload, steps, warmup, nested=False):
    """Timed and warmup steps: as given, else 50 and 5 (3 and 1 for the
    uneven batch, whose steps take seconds; nested, it runs 2 and 1)."""
    heavy = workload == "uneven"
    if heavy and nested:
        args.steps, args.warmup = 2, 1
        return
    args.steps = steps if steps is not None else (3 if heavy else 50)
    args.warmup = warmup if warmup is not None else (1 if heavy else 5)


def exact(line) -> bool:
    """Every oracle comparison in the line (and its nested lines) matched."""
    chk = line.get("oracle_check")
    if chk and chk["rows_matched"] != chk["rows_checked"]:
        return False
    dig = line.get("oracle_digest")
    if dig and not dig["match"]:
        return False
    if "error" in line:
        return False
    return all(exact(sub) for sub in line.get("configs", {}).values() if "skipped" not in sub)


if __name__ == "__main__":
    main()
