"""Writes tests/golden/uneven_oracle_digest.json: digests of the CPU oracle's
full answer on the uneven workload (10,000,000 objects x 64 dims, per-dim
Zipf(1.1) over 1,024 buckets, 16,384 queries of 4..512 range items, k = 100;
seed 1603083900 + 4).

The oracle's inverted-index search (Definition 2.1 counts, top-k in the
order count descending, id ascending) runs over every query, queries split
over host threads.  Stored: the SHA-256 of the whole answer (ids then counts,
little-endian uint32, row-major [16,384][100]), the SHA-256 of every block of
1,024 rows, and the total number of postings scanned.  Nothing here comes
from the GPU path; only `oracle` and the seeded generators are used.

Run from the repository root:  python tests/golden/make_oracle_digests.py
(about 40 minutes on 8 cores).
"""
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uneven_oracle_digest.json")
BLOCK = 1024


def answer_digest(ids: np.ndarray, cts: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(ids, dtype="<u4").tobytes())
    h.update(np.ascontiguousarray(cts, dtype="<u4").tobytes())
    return h.hexdigest()


def oracle_answer(values, V, queries, k, threads, chunk=8, progress=None):
    """O2 over every query of the batch, chunks of queries on host threads
    (the C search releases the interpreter lock)."""
    idx = oracle.build_csr(values, V)
    nq = queries.n_queries
    ids = np.zeros((nq, k), np.uint32)
    cts = np.zeros((nq, k), np.uint32)
    scanned = np.zeros(nq, np.uint64)

    def run(q0):
        q1 = min(nq, q0 + chunk)
        a, b, _, s = oracle.search_idx(idx, queries, k, q0, q1)
        ids[q0:q1], cts[q0:q1], scanned[q0:q1] = a, b, s
        return q1 - q0

    done = 0
    with cf.ThreadPoolExecutor(threads) as pool:
        for n in pool.map(run, range(0, nq, chunk)):
            done += n
            if progress and done % 512 < chunk:
                progress(done)
    return ids, cts, scanned


def main():
    t0 = time.time()
    inst = workloads.uneven()
    print("generated", round(time.time() - t0, 1), "s", flush=True)
    threads = os.cpu_count() or 1
    ids, cts, scanned = oracle_answer(
        inst.values, inst.V, inst.queries, inst.k, threads,
        progress=lambda d: print("queries done", d, round(time.time() - t0, 1), "s", flush=True))
    out = {
        "workload": "uneven: 10,000,000 objects x 64 dims, per-dim Zipf(1.1) over 1,024 "
                    "buckets; 16,384 queries of U{4..512} range items; k=100",
        "seed": workloads.BASE_SEED + workloads.CONFIG_IDS["uneven"],
        "n_objects": int(inst.n), "n_queries": int(inst.queries.n_queries), "k": int(inst.k),
        "layout": "sha256 of ids then counts, little-endian uint32, row-major [n_queries][k]",
        "sha256": answer_digest(ids, cts),
        "block_rows": BLOCK,
        "block_sha256": [answer_digest(ids[b:b + BLOCK], cts[b:b + BLOCK])
                         for b in range(0, inst.queries.n_queries, BLOCK)],
        "postings_scanned": int(scanned.sum()),
        "kth_count_mean": float(cts[:, inst.k - 1].mean()),
        "oracle_seconds": round(time.time() - t0, 1), "threads": threads,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
