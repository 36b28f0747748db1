"""CPU oracle for the match-count model, c-PQ and the LSH front-end.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never does, and
this package imports nothing from the GPU library.

Contents (each function names the passage of the paper it follows):

* ``brute_force_counts`` / ``brute_force_topk`` -- Definition 2.1 written out
  over every object (O1).
* ``build_csr`` / ``search_idx`` / ``match_counts`` -- the inverted-index scan
  with a count array and top-k selection, the shape of the paper's CPU-Idx
  baseline (Section 6.1.2), in plain C (O2).
* ``cpq_simulate`` -- Algorithm 1 (update on the Count Priority Queue,
  Section 3.3.1) run sequentially, with its trace (O3).
* ``lsh_signatures`` -- E2LSH (Equation of Section 4.2.3) followed by the
  re-hash r_i (Section 4.1.2), in float64 (O4).
* ``exact_knn_l2`` / ``recall`` / ``approximation_ratio`` -- exact l2
  neighbours and the approximation ratio of Section 6.4.1 (O5).
* ``oracle.rbh`` -- random binning hashing for the Laplacian kernel with its
  MurmurHash3 re-hash (Section 4.1.3).
* ``oracle.sequence`` -- sequence search with the Shotgun-and-Assembly
  scheme: ordered n-grams, top-K candidates, Algorithm 2 and the top-k
  certificate (Section 5.1); edit distance in plain C (edit_distance.c).

Answer order everywhere: count descending, then id ascending (the paper
breaks ties randomly; a fixed total order makes the answer unique).  Rows
list min(k, n) objects; slots past n hold (UINT32_MAX, 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "genie_oracle.c")
_SRC_ED = os.path.join(_HERE, "edit_distance.c")
_LIB = os.path.join(_HERE, "liboracle.so")
UINT32_MAX = 0xFFFFFFFF

_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Werror",
                               "-shared", "-fPIC", _SRC, _SRC_ED, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_build_csr.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.c_uint32, u64p, u32p]
        lib.oracle_search_idx.argtypes = [u64p, u32p, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, u64p, u32p, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint32, u32p, u32p,
                                          u32p, u64p]
        lib.oracle_match_counts.argtypes = [u64p, u32p, ctypes.c_uint64, ctypes.c_uint32,
                                            ctypes.c_uint32, u32p, ctypes.c_uint64, u32p,
                                            u64p]
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.oracle_edit_distance.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32]
        lib.oracle_edit_distance.restype = ctypes.c_uint32
        lib.oracle_edit_distances.argtypes = [u8p, u64p, u64p, u8p, u64p, u64p, ctypes.c_uint64,
                                              u32p]
        _lib = lib
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ----------------------------------------------------------------------------
# O1: Definition 2.1 over every object
# ----------------------------------------------------------------------------

def brute_force_counts(values: np.ndarray, items: np.ndarray) -> np.ndarray:
    """MC(Q, O) for every object O (Definition 2.1).

    values: [n, d] integers; items: [s, 3] (dim, lo, hi).  Item r contains the
    element (dim, v) of O iff lo <= v <= hi (Example 2.1, inclusive range), so
    C(r, O) is 0 or 1 and MC sums it over the items.
    """
    values = np.asarray(values)
    n = values.shape[0]
    counts = np.zeros(n, dtype=np.int64)
    for dim, lo, hi in np.asarray(items, dtype=np.int64).reshape(-1, 3):
        col = values[:, dim].astype(np.int64)
        counts += ((col >= lo) & (col <= hi)).astype(np.int64)
    return counts


def topk_from_counts(counts: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """The k first objects of the total order (count desc, id asc)."""
    counts = np.asarray(counts, dtype=np.int64)
    n = counts.shape[0]
    order = np.lexsort((np.arange(n), -counts))[:min(k, n)]
    ids = np.full(k, UINT32_MAX, dtype=np.uint32)
    cts = np.zeros(k, dtype=np.uint32)
    ids[:len(order)] = order.astype(np.uint32)
    cts[:len(order)] = counts[order].astype(np.uint32)
    return ids, cts


def brute_force_topk(values: np.ndarray, queries, k: int, qs=None):
    """O1 for a list of queries (workloads.Queries); returns ids, counts [nq, k]."""
    qs = range(queries.n_queries) if qs is None else list(qs)
    ids = np.zeros((len(qs), k), dtype=np.uint32)
    cts = np.zeros((len(qs), k), dtype=np.uint32)
    for r, q in enumerate(qs):
        ids[r], cts[r] = topk_from_counts(brute_force_counts(values, queries.items_of(q)), k)
    return ids, cts


# ----------------------------------------------------------------------------
# O2: inverted-index scan (CPU-Idx shape), plain C
# ----------------------------------------------------------------------------

class CsrIndex:
    """Keyword -> postings CSR built by the oracle (Section 3.2)."""

    def __init__(self, values: np.ndarray, V: int):
        values = np.ascontiguousarray(values, dtype=np.uint32)
        self.n, self.d = values.shape
        self.V = int(V)
        self.off = np.zeros(self.d * self.V + 1, dtype=np.uint64)
        self.post = np.zeros(max(1, self.n * self.d), dtype=np.uint32)
        rc = _load().oracle_build_csr(_p(values, ctypes.c_uint32), self.n, self.d, self.V,
                                      _p(self.off, ctypes.c_uint64),
                                      _p(self.post, ctypes.c_uint32))
        if rc != 0:
            raise ValueError(f"oracle_build_csr failed: {rc}")

    def postings(self, dim: int, v: int) -> np.ndarray:
        key = dim * self.V + v
        return self.post[int(self.off[key]):int(self.off[key + 1])]


def build_csr(values: np.ndarray, V: int) -> CsrIndex:
    return CsrIndex(values, V)


def search_idx(index: CsrIndex, queries, k: int, q_begin: int = 0,
               q_end: Optional[int] = None):
    """O2 over queries q_begin..q_end-1.

    Returns (ids [nq,k], counts [nq,k], kth [nq], scanned [nq]).
    Raises if an invariant of Definition 2.1 fails (sum of counts equals the
    postings scanned; no count above the number of items).
    """
    q_end = queries.n_queries if q_end is None else q_end
    nq = q_end - q_begin
    ids = np.zeros((max(nq, 0), k), dtype=np.uint32)
    cts = np.zeros((max(nq, 0), k), dtype=np.uint32)
    kth = np.zeros(max(nq, 0), dtype=np.uint32)
    scanned = np.zeros(max(nq, 0), dtype=np.uint64)
    if nq <= 0:
        return ids, cts, kth, scanned
    off = np.ascontiguousarray(queries.q_offsets, dtype=np.uint64)
    items = np.ascontiguousarray(queries.items, dtype=np.uint32).reshape(-1)
    if items.size == 0:
        items = np.zeros(3, dtype=np.uint32)
    rc = _load().oracle_search_idx(_p(index.off, ctypes.c_uint64), _p(index.post, ctypes.c_uint32),
                                   index.n, index.d, index.V, _p(off, ctypes.c_uint64),
                                   _p(items, ctypes.c_uint32), q_begin, q_end, k,
                                   _p(ids, ctypes.c_uint32), _p(cts, ctypes.c_uint32),
                                   _p(kth, ctypes.c_uint32), _p(scanned, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"oracle_search_idx failed: {rc}")
    return ids, cts, kth, scanned


def match_counts(index: CsrIndex, items: np.ndarray) -> Tuple[np.ndarray, int]:
    """Full MC vector of one query by index scan; returns (counts [n], scanned)."""
    items = np.ascontiguousarray(items, dtype=np.uint32).reshape(-1)
    n_items = items.size // 3
    if items.size == 0:
        items = np.zeros(3, dtype=np.uint32)
    out = np.zeros(max(index.n, 1), dtype=np.uint32)
    scanned = np.zeros(1, dtype=np.uint64)
    rc = _load().oracle_match_counts(_p(index.off, ctypes.c_uint64), _p(index.post, ctypes.c_uint32),
                                     index.n, index.d, index.V, _p(items, ctypes.c_uint32),
                                     n_items, _p(out, ctypes.c_uint32),
                                     _p(scanned, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"oracle_match_counts failed: {rc}")
    return out[:index.n], int(scanned[0])


# ----------------------------------------------------------------------------
# O3: Algorithm 1 run sequentially (Section 3.3.1)
# ----------------------------------------------------------------------------

class CpqTrace:
    """State of c-PQ after each scanned item of one query."""

    def __init__(self):
        self.steps: List[Dict] = []
        self.bc: Dict[int, int] = {}
        self.ht: Dict[int, int] = {}
        self.za: List[int] = []
        self.at: int = 1
        self.inserts: int = 0


def cpq_simulate(index: CsrIndex, items: np.ndarray, k: int) -> CpqTrace:
    """Algorithm 1 for one query, one posting at a time, in the order:
    items as given, keywords lo..hi of each item, postings ascending.

    Bitmap Counter BC (exact counts), Hash Table HT (id -> count), Gate =
    ZipperArray ZA (1-based, indices 1..maxc; this reading allocates index
    maxc+1 as a zero sentinel so that AT may reach maxc+1, as the worked
    example ends with AT = maxc + 1) and AuditThreshold AT starting at 1.
    maxc is the number of items (the largest possible count).

    Per posting O:  val = BC[O] + 1; BC[O] = val; if val >= AT: put (O, val)
    into HT, ZA[val] += 1, and while ZA[AT] >= k: AT += 1.
    """
    items = np.asarray(items, dtype=np.int64).reshape(-1, 3)
    maxc = len(items)
    tr = CpqTrace()
    tr.za = [0] * (maxc + 2)
    bc, ht, za = tr.bc, tr.ht, tr.za
    at = 1
    for dim, lo, hi in items:
        hi = min(hi, index.V - 1)
        for v in range(lo, hi + 1):
            for o in index.postings(int(dim), int(v)):
                o = int(o)
                val = bc.get(o, 0) + 1
                bc[o] = val
                if val >= at:
                    ht[o] = val
                    tr.inserts += 1
                    za[val] += 1
                    while za[at] >= k:
                        at += 1
        tr.steps.append({"bc": dict(bc), "ht": dict(ht), "za": list(za[1:maxc + 1]),
                         "at": at})
    tr.at = at
    return tr


# ----------------------------------------------------------------------------
# O4: E2LSH + re-hash in float64 (Section 4.1.2, Section 4.2.3)
# ----------------------------------------------------------------------------

def e2lsh_f64(points: np.ndarray, a: np.ndarray, b: np.ndarray, w: float,
              chunk_rows: int = 1 << 16) -> np.ndarray:
    """h_i(p) = floor((a_i . p + b_i) / w) in float64 (Section 4.2.3).

    a: [m, dim]; b: [m]; points: [n, dim].  The float32 inputs are widened to
    float64, where each product is exact; the floor is the mathematical one
    (toward minus infinity).  Returns int64 [n, m].
    """
    points = np.asarray(points)
    A = np.asarray(a, dtype=np.float64)
    B = np.asarray(b, dtype=np.float64)
    n = points.shape[0]
    out = np.empty((n, A.shape[0]), dtype=np.int64)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        proj = points[r0:r1].astype(np.float64) @ A.T
        out[r0:r1] = np.floor((proj + B) / np.float64(w)).astype(np.int64)
    return out


def rehash(h: np.ndarray, rehash_params: np.ndarray, log2_buckets: int) -> np.ndarray:
    """r_i(h) into [0, 2^log2_buckets) (Section 4.1.2, re-hashing).

    The paper asks for a random projection of the signature space onto D
    buckets with collision probability about 1/D.  This reading uses the
    multiply-add-shift universal hash: u = the 32-bit two's complement pattern
    of h zero-extended to 64 bits; r_i(u) = ((A_i * u + B_i) mod 2^64) >>
    (64 - log2 D), with A_i odd.  rehash_params = [A_0, B_0, A_1, B_1, ...].
    """
    h = np.asarray(h, dtype=np.int64)
    if np.any(h < -(2 ** 31)) or np.any(h >= 2 ** 31):
        raise OverflowError("LSH signature outside the int32 range")
    u = (h & 0xFFFFFFFF).astype(np.uint64)
    A = np.asarray(rehash_params, dtype=np.uint64)[0::2]
    Bv = np.asarray(rehash_params, dtype=np.uint64)[1::2]
    with np.errstate(over="ignore"):
        x = u * A[None, :] + Bv[None, :]
    return (x >> np.uint64(64 - log2_buckets)).astype(np.uint32)


def lsh_signatures(points, a, b, w, rehash_params, log2_buckets,
                   chunk_rows: int = 1 << 16) -> np.ndarray:
    """Object of Section 4.1.2: [r_1(h_1(p)), ..., r_m(h_m(p))], uint32 [n, m]."""
    n = np.asarray(points).shape[0]
    m = np.asarray(a).shape[0]
    out = np.empty((n, m), dtype=np.uint32)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        out[r0:r1] = rehash(e2lsh_f64(points[r0:r1], a, b, w, chunk_rows),
                            rehash_params, log2_buckets)
    return out


# ----------------------------------------------------------------------------
# O5: exact l2 neighbours, recall and approximation ratio (Section 6.4.1)
# ----------------------------------------------------------------------------

def exact_knn_l2(points: np.ndarray, queries: np.ndarray, k: int,
                 qchunk: int = 256) -> Tuple[np.ndarray, np.ndarray]:
    """Exact k nearest neighbours by float64 l2 distance, ties by id.

    Returns (ids [nq, k], dist [nq, k]) sorted ascending.
    """
    P = np.asarray(points, dtype=np.float64)
    pn = np.einsum("ij,ij->i", P, P)
    nq = queries.shape[0]
    ids = np.zeros((nq, k), dtype=np.int64)
    dist = np.zeros((nq, k), dtype=np.float64)
    for q0 in range(0, nq, qchunk):
        q1 = min(nq, q0 + qchunk)
        Q = np.asarray(queries[q0:q1], dtype=np.float64)
        d2 = pn[None, :] - 2.0 * (Q @ P.T) + np.einsum("ij,ij->i", Q, Q)[:, None]
        np.maximum(d2, 0.0, out=d2)
        for r in range(q1 - q0):
            # every point at or below the k-th smallest distance, then the
            # order (distance, id): points tied at the k-th distance are
            # taken by id
            kth = np.partition(d2[r], k - 1)[k - 1]
            cand = np.flatnonzero(d2[r] <= kth)
            order = np.lexsort((cand, d2[r, cand]))[:k]
            ids[q0 + r] = cand[order]
            dist[q0 + r] = np.sqrt(d2[r, cand[order]])
    return ids, dist


def recall(found_ids: np.ndarray, true_ids: np.ndarray) -> float:
    """Fraction of the true k neighbours present in the returned k."""
    hit = 0
    for f, t in zip(found_ids, true_ids):
        hit += len(set(int(x) for x in f) & set(int(x) for x in t))
    return hit / float(true_ids.size)


def approximation_ratio(points: np.ndarray, queries: np.ndarray, found_ids: np.ndarray,
                        true_dist: np.ndarray) -> float:
    """(1/k) sum_i ||p_i - q|| / ||p*_i - q|| with both lists sorted by distance
    (Section 6.4.1), averaged over queries; pairs with a zero true distance
    are skipped."""
    ratios = []
    for q, f, td in zip(queries, found_ids, true_dist):
        fp = np.asarray(points[f], dtype=np.float64)
        fd = np.sort(np.sqrt(((fp - np.asarray(q, dtype=np.float64)) ** 2).sum(axis=1)))
        ok = td > 0
        if np.any(ok):
            ratios.append(np.mean(fd[ok] / td[ok]))
    return float(np.mean(ratios)) if ratios else float("nan")
