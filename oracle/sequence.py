"""CPU oracle for similarity search on sequences under edit distance with the
Shotgun-and-Assembly scheme (Section 5.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``ordered_ngrams`` -- G(S) of Section 5.1.1: for every window position p of
  a length-n sliding window, the pair (S[p:p+n], i) where i is the number of
  earlier windows holding the same n-gram (Example 5.1).
* ``mc_ordered`` -- MC(G(S), G(Q)) = |G(S) and G(Q)|: the match count of
  Definition 2.1 when every element of G(Q) is one single-keyword item and
  every element of G(S) one keyword of the object.
* ``mc_by_counts`` -- Lemma 5.1's closed form, sum over n-grams of
  min(c_s, c_q).  The pins check it against ``mc_ordered``; the corpus-wide
  counts below use it.
* ``edit_distance`` / ``edit_distances`` -- Levenshtein distance, by the
  textbook dynamic programme in plain C (edit_distance.c).
* ``SeqCorpus`` -- the data sequences and, per query, the match count of
  every sequence (Lemma 5.1 over the windows that hold one of the query's
  n-grams) and the top-K candidates in the total order (count desc, id asc).
* ``verify`` -- Algorithm 2 (verification), generalised from the most
  similar sequence to the k most similar: the answer is kept as the k best
  (distance, candidate position) pairs, tau_k' is the k-th best distance
  (infinite until k candidates are verified), the filtering bound is
  theta = |Q| - n + 1 - n (tau_k' - 1), the scan of the candidates in count
  order stops at the first candidate whose count is below theta, and a
  candidate with |Q| - |S| > tau_k' is skipped.  With k = 1 these are the
  steps of Algorithm 2 exactly.  Ties in distance go to the earlier
  candidate (a later one must be strictly closer to replace it).
* ``certified`` -- Theorem 5.2: the answer is the true top-k of the whole
  data set when c_K < |Q| - n + 1 - tau_k' n, c_K being the count of the
  K-th candidate; and trivially when the candidates are every sequence.
* ``sequence_search`` -- decomposition, top-K, Algorithm 2 and the
  certificate for a batch of queries.
"""
from __future__ import annotations

import ctypes
from collections import Counter
from typing import List, Sequence, Tuple

import numpy as np

from . import UINT32_MAX, _load, _p, topk_from_counts


def ordered_ngrams(s: bytes, n: int) -> List[Tuple[bytes, int]]:
    """G(S) in window order (Section 5.1.1, Example 5.1)."""
    seen = {}
    out = []
    for p in range(len(s) - n + 1):
        g = bytes(s[p:p + n])
        i = seen.get(g, 0)
        out.append((g, i))
        seen[g] = i + 1
    return out


def mc_ordered(s: bytes, q: bytes, n: int) -> int:
    """|G(S) and G(Q)|: the number of ordered n-grams the two share."""
    return len(set(ordered_ngrams(s, n)) & set(ordered_ngrams(q, n)))


def mc_by_counts(s: bytes, q: bytes, n: int) -> int:
    """Lemma 5.1: sum over distinct n-grams g of min(c_s(g), c_q(g))."""
    cs = Counter(bytes(s[p:p + n]) for p in range(len(s) - n + 1))
    cq = Counter(bytes(q[p:p + n]) for p in range(len(q) - n + 1))
    return sum(min(c, cs[g]) for g, c in cq.items())


def edit_distance(a: bytes, b: bytes) -> int:
    a = np.frombuffer(bytes(a), dtype=np.uint8)
    b = np.frombuffer(bytes(b), dtype=np.uint8)
    if a.size == 0 or b.size == 0:
        return int(max(a.size, b.size))
    u8p = ctypes.c_uint8
    d = _load().oracle_edit_distance(_p(np.ascontiguousarray(a), u8p), a.size,
                                     _p(np.ascontiguousarray(b), u8p), b.size)
    if d == UINT32_MAX:
        raise MemoryError("oracle_edit_distance")
    return int(d)


def edit_distances(a_chars, a_off, ai, b_chars, b_off, bi) -> np.ndarray:
    """Distances of the pairs (a-sequence ai[p], b-sequence bi[p])."""
    a_chars = np.ascontiguousarray(a_chars, dtype=np.uint8)
    b_chars = np.ascontiguousarray(b_chars, dtype=np.uint8)
    if a_chars.size == 0:
        a_chars = np.zeros(1, np.uint8)
    if b_chars.size == 0:
        b_chars = np.zeros(1, np.uint8)
    a_off = np.ascontiguousarray(a_off, dtype=np.uint64)
    b_off = np.ascontiguousarray(b_off, dtype=np.uint64)
    ai = np.ascontiguousarray(ai, dtype=np.uint64)
    bi = np.ascontiguousarray(bi, dtype=np.uint64)
    out = np.zeros(max(1, ai.size), dtype=np.uint32)
    rc = _load().oracle_edit_distances(_p(a_chars, ctypes.c_uint8), _p(a_off, ctypes.c_uint64),
                                       _p(ai, ctypes.c_uint64), _p(b_chars, ctypes.c_uint8),
                                       _p(b_off, ctypes.c_uint64), _p(bi, ctypes.c_uint64),
                                       ai.size, _p(out, ctypes.c_uint32))
    if rc != 0:
        raise MemoryError("oracle_edit_distances")
    return out[:ai.size]


def _window_codes(chars: np.ndarray, starts: np.ndarray, n: int) -> np.ndarray:
    """The n bytes of every window, packed big-endian into one integer."""
    code = np.zeros(starts.size, dtype=np.uint64)
    for i in range(n):
        code = (code << np.uint64(8)) | chars[starts + i].astype(np.uint64)
    return code


class SeqCorpus:
    """Data sequences (bytes back to back, offsets [n+1]) and their windows."""

    def __init__(self, chars: np.ndarray, offsets: np.ndarray, n: int):
        if not 1 <= n <= 8:
            raise ValueError("n-gram length must be 1..8")
        self.chars = np.ascontiguousarray(chars, dtype=np.uint8)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.n = int(n)
        self.N = self.offsets.size - 1
        lens = np.diff(self.offsets).astype(np.int64)
        self.lens = lens
        w = np.maximum(lens - n + 1, 0)
        seq = np.repeat(np.arange(self.N, dtype=np.int64), w)
        first = np.cumsum(w) - w
        pos = np.arange(seq.size, dtype=np.int64) - first[seq]
        starts = self.offsets[:-1].astype(np.int64)[seq] + pos
        self.window_seq = seq
        self.window_code = _window_codes(self.chars, starts, n)

    def seq(self, i: int) -> bytes:
        return self.chars[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def match_counts(self, q: bytes) -> np.ndarray:
        """MC(G(S), G(Q)) for every sequence S (Lemma 5.1)."""
        n = self.n
        cq = Counter(_window_codes(np.frombuffer(bytes(q), np.uint8),
                                   np.arange(max(len(q) - n + 1, 0)), n).tolist())
        counts = np.zeros(self.N, dtype=np.int64)
        if not cq:
            return counts
        codes = np.array(sorted(cq), dtype=np.uint64)
        mask = np.isin(self.window_code, codes)
        seq = self.window_seq[mask]
        which = np.searchsorted(codes, self.window_code[mask])
        # c_s per (sequence, n-gram of Q)
        pair = seq * codes.size + which
        upair, cs = np.unique(pair, return_counts=True)
        cq_arr = np.array([cq[int(c)] for c in codes], dtype=np.int64)
        np.add.at(counts, upair // codes.size, np.minimum(cs, cq_arr[upair % codes.size]))
        return counts

    def candidates(self, q: bytes, K: int) -> Tuple[np.ndarray, np.ndarray]:
        """Top-K by (count desc, id asc); slots past N hold (UINT32_MAX, 0)."""
        return topk_from_counts(self.match_counts(q), K)


def verify(q: bytes, cand_ids: np.ndarray, cand_counts: np.ndarray,
           seq_of, n: int, k: int = 1) -> Tuple[List[int], List[int]]:
    """Algorithm 2 over candidates in count order, for the k most similar.

    seq_of(id) returns the sequence; ids equal to UINT32_MAX are empty slots.
    Returns (positions, distances) of the answer, best first.
    """
    Q = len(q)
    best: List[Tuple[int, int]] = []        # (distance, candidate position), sorted

    def tau_k() -> float:
        return best[k - 1][0] if len(best) >= k else float("inf")

    for j in range(len(cand_ids)):
        cid = int(cand_ids[j])
        if cid == UINT32_MAX:
            break
        if len(best) >= k:
            theta = Q - n + 1 - n * (tau_k() - 1)      # filtering bound
            if theta > int(cand_counts[j]):
                break                                  # Theorem 5.1: no closer one left
            s = seq_of(cid)
            if Q - len(s) > tau_k():                   # length filter
                continue
        else:
            s = seq_of(cid)
        t = edit_distance(q, s)
        if len(best) < k or t < tau_k():
            best.append((t, j))
            best.sort()
            del best[k:]
    return [j for _, j in best], [t for t, _ in best]


def certified(q_len: int, n: int, cand_ids: np.ndarray, cand_counts: np.ndarray,
              dists: Sequence[int], k: int, n_objects: int) -> bool:
    """Theorem 5.2 for one query (K = len(cand_ids))."""
    K = len(cand_ids)
    if K >= n_objects:
        return True                     # every sequence was a candidate
    if len(dists) < k:
        return False
    c_K = int(cand_counts[K - 1])
    return c_K < q_len - n + 1 - int(dists[k - 1]) * n


class SeqAnswer:
    def __init__(self, nq: int, k: int, K: int):
        self.ids = np.full((nq, k), UINT32_MAX, dtype=np.uint32)
        self.dist = np.full((nq, k), UINT32_MAX, dtype=np.uint32)
        self.cert = np.zeros(nq, dtype=np.uint32)
        self.cand_ids = np.zeros((nq, K), dtype=np.uint32)
        self.cand_counts = np.zeros((nq, K), dtype=np.uint32)


def sequence_search(corpus: SeqCorpus, qchars: np.ndarray, qoffsets: np.ndarray,
                    K: int, k: int, queries=None) -> SeqAnswer:
    """Top-K candidates, Algorithm 2 and Theorem 5.2 for queries (default: all)."""
    qoffsets = np.asarray(qoffsets, dtype=np.uint64)
    qs = range(qoffsets.size - 1) if queries is None else list(queries)
    ans = SeqAnswer(len(qs), k, K)
    for r, qi in enumerate(qs):
        q = np.asarray(qchars[int(qoffsets[qi]):int(qoffsets[qi + 1])], np.uint8).tobytes()
        ids, cts = corpus.candidates(q, K)
        ans.cand_ids[r], ans.cand_counts[r] = ids, cts
        pos, dist = verify(q, ids, cts, corpus.seq, corpus.n, k)
        for t, (j, d) in enumerate(zip(pos, dist)):
            ans.ids[r, t] = ids[j]
            ans.dist[r, t] = d
        ans.cert[r] = certified(len(q), corpus.n, ids, cts, dist, k, corpus.N)
    return ans
