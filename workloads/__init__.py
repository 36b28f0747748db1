"""Seeded synthetic inputs for the match-count workloads.

This module is the only code shared by the CPU oracle's tests and the GPU
path.  It draws random numbers and lays them out; it holds none of the
method's arithmetic (no counting, no hashing, no selection).

Workloads (the paper's datasets are not available; these stand in for them):

* ``tiny``        10,000 objects x 16 dims, values uniform in [0, 64); 100
                  queries of one item per dim, [v-2, v+2] around a random
                  object's value; k = 10.
* ``relational``  1,000,000 x 32 dims, 256 buckets, per-dim finite Zipf(1.1)
                  (P(b) proportional to (b+1)^-1.1, bucket 0 is the head);
                  1,024 queries, one range item per dim centred on a random
                  object's value with width uniform in {0..8}; k = 100.
                  Stands in for the Adult relational table (Section 6.1.1).
* ``ann``         1,000,000 float32 points in 128-d from a 64-component
                  Gaussian mixture clipped at 0; 4,096 perturbed queries;
                  237 E2LSH functions (w = 4.0) re-hashed into 8,192 buckets;
                  k = 100.  Stands in for SIFT (Section 6.1.1).
* ``uneven``      10,000,000 x 64 dims, 1,024 buckets, Zipf(1.1); 16,384
                  queries with 4..512 items each; k = 100.
* ``laplace``     the ``ann`` points through RBH functions for the Laplacian
                  kernel (Section 4.1.3); stands in for OCR.
* ``sequence``    5,000,000 title-like strings (words of a Zipf vocabulary
                  joined by spaces); 1,024 queries of 40 characters, each a
                  data string with 20 % of its characters replaced; 3-grams,
                  K = 32 candidates, k = 1.  Stands in for DBLP titles
                  (Sections 5.1 and 6.1.1).

Every generator takes explicit sizes so that tests can draw scaled-down
instances with the same structure.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

BASE_SEED = 1603083900
CONFIG_IDS = {"tiny": 1, "relational": 2, "ann": 3, "uneven": 4, "serving": 5, "laplace": 6,
              "sequence": 7}


def rng_streams(config_id: int, salt: int = 0):
    """Independent child generators (objects, queries, lsh) for one workload."""
    ss = np.random.SeedSequence(BASE_SEED + config_id + salt)
    return [np.random.default_rng(s) for s in ss.spawn(3)]


# ----------------------------------------------------------------------------
# value distributions
# ----------------------------------------------------------------------------

def zipf_cdf(V: int, a: float = 1.1) -> np.ndarray:
    """CDF of the finite Zipf law P(b) ~ (b+1)^-a on b in [0, V)."""
    w = np.arange(1, V + 1, dtype=np.float64) ** (-a)
    c = np.cumsum(w)
    return c / c[-1]


def objects_uniform(rng, n: int, d: int, V: int) -> np.ndarray:
    return rng.integers(0, V, size=(n, d), dtype=np.uint32)


def objects_zipf(rng, n: int, d: int, V: int, a: float = 1.1,
                 chunk_rows: int = 1 << 20) -> np.ndarray:
    """Independent per-dim finite Zipf values, drawn by inverse CDF."""
    cdf = zipf_cdf(V, a)
    out = np.empty((n, d), dtype=np.uint32)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        u = rng.random((r1 - r0, d))
        idx = np.searchsorted(cdf, u, side="right")
        np.minimum(idx, V - 1, out=idx)
        out[r0:r1] = idx.astype(np.uint32)
    return out


# ----------------------------------------------------------------------------
# query layouts: CSR of items, each item = (dim, lo, hi) inclusive
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Queries:
    q_offsets: np.ndarray  # uint64 [nq+1]
    items: np.ndarray      # uint32 [n_items, 3] (dim, lo, hi)

    @property
    def n_queries(self) -> int:
        return len(self.q_offsets) - 1

    def items_of(self, q: int) -> np.ndarray:
        return self.items[self.q_offsets[q]:self.q_offsets[q + 1]]

    def max_items(self) -> int:
        if self.n_queries == 0:
            return 0
        return int(np.max(np.diff(self.q_offsets.astype(np.int64))))

    def subset(self, qs) -> "Queries":
        qs = list(qs)
        lens = [int(self.q_offsets[q + 1] - self.q_offsets[q]) for q in qs]
        off = np.zeros(len(qs) + 1, dtype=np.uint64)
        off[1:] = np.cumsum(lens, dtype=np.uint64)
        if qs:
            items = np.concatenate([self.items_of(q) for q in qs]).astype(np.uint32)
        else:
            items = np.zeros((0, 3), dtype=np.uint32)
        return Queries(off, items.reshape(-1, 3))


def queries_halfwidth(rng, values: np.ndarray, V: int, nq: int, half: int) -> Queries:
    """One item per dim: [v-half, v+half] clipped, v = a random object's value."""
    n, d = values.shape
    objs = rng.integers(0, n, size=nq)
    c = values[objs].astype(np.int64)                       # [nq, d]
    lo = np.clip(c - half, 0, V - 1)
    hi = np.clip(c + half, 0, V - 1)
    dims = np.broadcast_to(np.arange(d, dtype=np.int64), (nq, d))
    items = np.stack([dims, lo, hi], axis=-1).reshape(-1, 3).astype(np.uint32)
    off = (np.arange(nq + 1, dtype=np.uint64) * np.uint64(d))
    return Queries(off, items)


def queries_random_width(rng, values: np.ndarray, V: int, nq: int, wmax: int = 8) -> Queries:
    """One item per dim centred on one random object's value per query.

    Width w ~ U{0..wmax} per item; lo = c - floor(w/2), hi = lo + w, clipped.
    """
    n, d = values.shape
    objs = rng.integers(0, n, size=nq)
    c = values[objs].astype(np.int64)
    w = rng.integers(0, wmax + 1, size=(nq, d))
    lo = c - w // 2
    hi = lo + w
    lo = np.clip(lo, 0, V - 1)
    hi = np.clip(hi, 0, V - 1)
    dims = np.broadcast_to(np.arange(d, dtype=np.int64), (nq, d))
    items = np.stack([dims, lo, hi], axis=-1).reshape(-1, 3).astype(np.uint32)
    off = (np.arange(nq + 1, dtype=np.uint64) * np.uint64(d))
    return Queries(off, items)


def queries_uneven(rng, values: np.ndarray, V: int, nq: int, smin: int = 4,
                   smax: int = 512, wmax: int = 8) -> Queries:
    """s ~ U{smin..smax} items per query; item j is on dim j mod d, centred on
    an independently drawn random object's value, width as above."""
    n, d = values.shape
    s = rng.integers(smin, smax + 1, size=nq)
    off = np.zeros(nq + 1, dtype=np.uint64)
    off[1:] = np.cumsum(s, dtype=np.uint64)
    total = int(off[-1])
    j = np.arange(total, dtype=np.int64) - np.repeat(off[:-1].astype(np.int64), s)
    dims = j % d
    objs = rng.integers(0, n, size=total)
    c = values[objs, dims].astype(np.int64)
    w = rng.integers(0, wmax + 1, size=total)
    lo = np.clip(c - w // 2, 0, V - 1)
    hi = np.clip(c - w // 2 + w, 0, V - 1)
    items = np.stack([dims, lo, hi], axis=-1).astype(np.uint32)
    return Queries(off, items)


def queries_exact(sig: np.ndarray) -> Queries:
    """Item i = (i, sig[i], sig[i]) for every hash function i of each query."""
    nq, m = sig.shape
    dims = np.broadcast_to(np.arange(m, dtype=np.uint32), (nq, m))
    items = np.stack([dims, sig, sig], axis=-1).reshape(-1, 3).astype(np.uint32)
    off = np.arange(nq + 1, dtype=np.uint64) * np.uint64(m)
    return Queries(off, items)


# ----------------------------------------------------------------------------
# relational-style workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Relational:
    name: str
    values: np.ndarray     # uint32 [n, d], each < V
    V: int
    queries: Queries
    k: int

    @property
    def n(self) -> int:
        return self.values.shape[0]

    @property
    def d(self) -> int:
        return self.values.shape[1]


def tiny(n: int = 10_000, d: int = 16, V: int = 64, nq: int = 100, k: int = 10,
         half: int = 2, salt: int = 0) -> Relational:
    ro, rq, _ = rng_streams(CONFIG_IDS["tiny"], salt)
    values = objects_uniform(ro, n, d, V)
    return Relational("tiny", values, V, queries_halfwidth(rq, values, V, nq, half), k)


def relational(n: int = 1_000_000, d: int = 32, V: int = 256, nq: int = 1024,
               k: int = 100, wmax: int = 8, a: float = 1.1, salt: int = 0) -> Relational:
    ro, rq, _ = rng_streams(CONFIG_IDS["relational"], salt)
    values = objects_zipf(ro, n, d, V, a)
    return Relational("relational", values, V, queries_random_width(rq, values, V, nq, wmax), k)


def uneven(n: int = 10_000_000, d: int = 64, V: int = 1024, nq: int = 16_384,
           k: int = 100, smin: int = 4, smax: int = 512, wmax: int = 8,
           a: float = 1.1, salt: int = 0) -> Relational:
    ro, rq, _ = rng_streams(CONFIG_IDS["uneven"], salt)
    values = objects_zipf(ro, n, d, V, a)
    return Relational("uneven", values, V,
                      queries_uneven(rq, values, V, nq, smin, smax, wmax), k)


# ----------------------------------------------------------------------------
# tau-ANN workload: raw points and LSH parameters (hashing is done elsewhere)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class AnnInputs:
    points: np.ndarray     # float32 [n, dim]
    queries: np.ndarray    # float32 [nq, dim]
    a: np.ndarray          # float32 [m, dim]   projection vectors, N(0, 1)
    b: np.ndarray          # float32 [m]        offsets, U[0, w)
    w: float
    rehash: np.ndarray     # uint64 [2m]        (A_i odd, B_i) interleaved
    log2_buckets: int
    k: int


def ann(n: int = 1_000_000, dim: int = 128, nq: int = 4096, m: int = 237,
        w: float = 4.0, log2_buckets: int = 13, components: int = 64,
        sigma: float = 0.5, qsigma: float = 0.1, k: int = 100,
        salt: int = 0, chunk_rows: int = 1 << 18) -> AnnInputs:
    ro, rq, rl = rng_streams(CONFIG_IDS["ann"], salt)
    points = gmm_points(ro, n, dim, components, sigma, chunk_rows)
    queries = ann_queries(rq, points, nq, qsigma)
    a = rl.standard_normal((m, dim), dtype=np.float32)
    b = rl.uniform(0.0, w, size=m).astype(np.float32)
    b = np.minimum(b, np.nextafter(np.float32(w), np.float32(0)))
    A = rl.integers(0, 2**63, size=m, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    B = rl.integers(0, 2**63, size=m, dtype=np.uint64) * np.uint64(2) + \
        rl.integers(0, 2, size=m, dtype=np.uint64)
    rehash = np.empty(2 * m, dtype=np.uint64)
    rehash[0::2] = A
    rehash[1::2] = B
    return AnnInputs(points, queries, a, b, float(w), rehash, int(log2_buckets), k)


def gmm_points(rng, n: int, dim: int, components: int = 64, sigma: float = 0.5,
               chunk_rows: int = 1 << 18) -> np.ndarray:
    """Equal-weight Gaussian mixture: means U[0, 8)^dim, per-coordinate sigma,
    clipped at 0 (non-negative features)."""
    means = rng.uniform(0.0, 8.0, size=(components, dim)).astype(np.float32)
    points = np.empty((n, dim), dtype=np.float32)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        comp = rng.integers(0, components, size=r1 - r0)
        x = means[comp] + np.float32(sigma) * rng.standard_normal((r1 - r0, dim), dtype=np.float32)
        np.maximum(x, 0.0, out=x)
        points[r0:r1] = x
    return points


@dataclasses.dataclass
class LaplaceInputs:
    points: np.ndarray     # float32 [n, dim]
    queries: np.ndarray    # float32 [nq, dim]
    g: np.ndarray          # float32 [m, dim] grid pitch per function and dimension
    u: np.ndarray          # float32 [m, dim] grid shift, in [0, g)
    seeds: np.ndarray      # uint32 [m] MurmurHash3 seed per function
    sigma: float
    log2_buckets: int
    k: int


def rbh_params(rng, m: int, dim: int, sigma: float):
    """Random binning functions for the Laplacian kernel exp(-||.||_1 / sigma):
    pitch ~ Gamma(2, sigma) and shift ~ U[0, pitch) per function and
    dimension, and a 32-bit re-hash seed per function."""
    g = rng.gamma(2.0, sigma, size=(m, dim)).astype(np.float32)
    g = np.maximum(g, np.float32(1e-6))
    u = (rng.random((m, dim)) * g).astype(np.float32)
    u = np.minimum(u, np.nextafter(g, np.float32(0)))
    seeds = rng.integers(0, 2**32, size=m, dtype=np.uint64).astype(np.uint32)
    return g, u, seeds


def laplace(n: int = 1_000_000, dim: int = 128, nq: int = 4096, m: int = 237,
            sigma: float = 32.0, log2_buckets: int = 13, components: int = 64,
            csigma: float = 0.5, qsigma: float = 0.1, k: int = 100, salt: int = 0,
            chunk_rows: int = 1 << 18) -> LaplaceInputs:
    """ANN in the Laplacian kernel space (Section 4.1.3): the Gaussian-mixture
    points of ``ann`` searched through m RBH functions re-hashed into
    2^log2_buckets buckets.  Stands in for the OCR workload of the paper."""
    ro, rq, rl = rng_streams(CONFIG_IDS["laplace"], salt)
    points = gmm_points(ro, n, dim, components, csigma, chunk_rows)
    queries = ann_queries(rq, points, nq, qsigma)
    g, u, seeds = rbh_params(rl, m, dim, sigma)
    return LaplaceInputs(points, queries, g, u, seeds, float(sigma), int(log2_buckets), k)


def ann_queries(rng, points: np.ndarray, nq: int, qsigma: float = 0.1) -> np.ndarray:
    """Queries = random data points + N(0, qsigma^2) per coordinate, clipped at 0."""
    n, dim = points.shape
    src = rng.integers(0, n, size=nq)
    q = points[src] + np.float32(qsigma) * rng.standard_normal((nq, dim), dtype=np.float32)
    np.maximum(q, 0.0, out=q)
    return q.astype(np.float32)


def random_small(rng, n: int, d: int, V: int, nq: int, max_items: int,
                 allow_empty: bool = True) -> Relational:
    """Tiny adversarial instances: random items on random dims (dims may
    repeat, ranges may overlap, be empty after clipping or exceed [0, V))."""
    values = rng.integers(0, V, size=(n, d), dtype=np.uint32)
    lens = rng.integers(0 if allow_empty else 1, max_items + 1, size=nq)
    off = np.zeros(nq + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens, dtype=np.uint64)
    total = int(off[-1])
    dims = rng.integers(0, d, size=total)
    lo = rng.integers(0, V + 2, size=total)
    hi = rng.integers(0, V + 2, size=total)
    # hi may be below lo (empty item) and either bound may lie past V-1
    items = np.stack([dims, lo, hi], axis=-1).astype(np.uint32).reshape(-1, 3)
    return Relational("random_small", values, V, Queries(off, items), 1)


# ----------------------------------------------------------------------------
# sequences (Section 5.1): title-like synthetic text
# ----------------------------------------------------------------------------

def pack_sequences(seqs) -> tuple:
    """bytes objects -> (chars uint8 [total], offsets uint64 [n+1])."""
    lens = np.array([len(x) for x in seqs], dtype=np.uint64)
    off = np.zeros(len(seqs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens, dtype=np.uint64)
    chars = np.frombuffer(b"".join(bytes(x) for x in seqs), dtype=np.uint8).copy()
    return chars, off


@dataclasses.dataclass
class SequenceInputs:
    chars: np.ndarray      # uint8: data sequences back to back
    offsets: np.ndarray    # uint64 [n+1]
    qchars: np.ndarray     # uint8: queries back to back
    qoffsets: np.ndarray   # uint64 [nq+1]
    sources: np.ndarray    # int64 [nq]: the data sequence each query was made from
    gram: int              # n of the n-grams
    K: int                 # candidates taken by match count
    k: int                 # answers after verification

    @property
    def n(self) -> int:
        return self.offsets.size - 1

    @property
    def nq(self) -> int:
        return self.qoffsets.size - 1

    def seq(self, i: int) -> bytes:
        return self.chars[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def query(self, j: int) -> bytes:
        return self.qchars[int(self.qoffsets[j]):int(self.qoffsets[j + 1])].tobytes()


TEXT_ALPHABET = b"abcdefghijklmnopqrstuvwxyz0123456789"


def text_vocabulary(rng, n_words: int, letter_a: float = 0.9):
    """Pseudo-words: letters drawn from a skewed law (P(letter of rank r) ~
    (r+1)^-letter_a over a seeded order of the 26 letters, digits rare),
    lengths 2..12 with the shortest words at the most frequent ranks."""
    letters = np.frombuffer(TEXT_ALPHABET[:26], np.uint8)[rng.permutation(26)]
    sym = np.concatenate([letters, np.frombuffer(TEXT_ALPHABET[26:], np.uint8)])
    w = np.concatenate([np.arange(1, 27, dtype=np.float64) ** (-letter_a),
                        np.full(10, 0.004)])
    cdf = np.cumsum(w / w.sum())
    lens = np.sort(2 + rng.binomial(10, 0.5, size=n_words)).astype(np.int64)
    off = np.zeros(n_words + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    idx = np.minimum(np.searchsorted(cdf, rng.random(int(off[-1])), side="right"), sym.size - 1)
    return sym[idx], off


def text_corpus(rng, n: int, vocab: int = 30_000, word_a: float = 1.0, wmin: int = 4,
                wmax: int = 14, chunk: int = 250_000):
    """n strings of wmin..wmax words (Zipf(word_a) over the vocabulary ranks)
    joined by single spaces."""
    vchars, voff = text_vocabulary(rng, vocab)
    vlen = np.diff(voff)
    wcdf = np.cumsum(np.arange(1, vocab + 1, dtype=np.float64) ** (-word_a))
    wcdf /= wcdf[-1]
    parts, lens_all = [], []
    for r0 in range(0, n, chunk):
        c = min(chunk, n - r0)
        nw = rng.integers(wmin, wmax + 1, size=c)
        words = np.minimum(np.searchsorted(wcdf, rng.random(int(nw.sum())), side="right"),
                           vocab - 1)
        wl = vlen[words] + 1                      # the word and one space after it
        total = int(wl.sum())
        rep = np.repeat(np.arange(words.size), wl)
        wstart = np.cumsum(wl) - wl
        inword = np.arange(total, dtype=np.int64) - wstart[rep]
        src = voff[words][rep] + np.minimum(inword, vlen[words][rep] - 1)
        out = np.where(inword == vlen[words][rep], np.uint8(ord(" ")), vchars[src])
        # drop the space after the last word of every string
        seq_end = np.cumsum(np.add.reduceat(wl, np.cumsum(nw) - nw))
        keep = np.ones(total, dtype=bool)
        keep[seq_end - 1] = False
        parts.append(out[keep].astype(np.uint8))
        lens_all.append(np.add.reduceat(wl, np.cumsum(nw) - nw) - 1)
    lens = np.concatenate(lens_all).astype(np.uint64)
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens, dtype=np.uint64)
    return np.concatenate(parts), off


def modified_queries(rng, chars: np.ndarray, offsets: np.ndarray, nq: int, qlen: int,
                     frac: float, alphabet: bytes = TEXT_ALPHABET + b" "):
    """nq data strings of exactly qlen characters, each with round(frac * qlen)
    distinct positions replaced by a different symbol of the alphabet."""
    lens = np.diff(offsets).astype(np.int64)
    pool = np.flatnonzero(lens == qlen)
    if pool.size < nq:
        raise ValueError(f"only {pool.size} strings of length {qlen}")
    src = rng.choice(pool, size=nq, replace=False)
    q = chars[offsets[src].astype(np.int64)[:, None] + np.arange(qlen)].copy()
    m = int(round(frac * qlen))
    alpha = np.frombuffer(alphabet, np.uint8)
    lut = np.full(256, 0, dtype=np.int64)
    lut[alpha] = np.arange(alpha.size)
    if m:
        pos = np.argsort(rng.random((nq, qlen)), axis=1)[:, :m]
        rows = np.arange(nq)[:, None]
        old = lut[q[rows, pos]]
        new = (old + 1 + rng.integers(0, alpha.size - 1, size=old.shape)) % alpha.size
        q[rows, pos] = alpha[new]
    qoff = np.arange(nq + 1, dtype=np.uint64) * np.uint64(qlen)
    return q.reshape(-1).astype(np.uint8), qoff, src.astype(np.int64)


def sequence(n: int = 5_000_000, nq: int = 1024, qlen: int = 40, frac: float = 0.2,
             gram: int = 3, K: int = 32, k: int = 1, salt: int = 0) -> SequenceInputs:
    """Sequence search under edit distance (Section 5.1) on title-like text;
    stands in for the DBLP titles of Section 6.1.1."""
    ro, rq, _ = rng_streams(CONFIG_IDS["sequence"], salt)
    chars, off = text_corpus(ro, n)
    qc, qo, src = modified_queries(rq, chars, off, nq, qlen, frac)
    return SequenceInputs(chars, off, qc, qo, src, gram, K, k)


def random_sequences(rng, n: int, alphabet: bytes, lmin: int, lmax: int):
    """Adversarial strings: i.i.d. symbols of a small alphabet (many repeated
    n-grams), lengths uniform in [lmin, lmax] (0 allowed)."""
    lens = rng.integers(lmin, lmax + 1, size=n)
    alpha = np.frombuffer(alphabet, np.uint8)
    chars = alpha[rng.integers(0, alpha.size, size=int(lens.sum()))]
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens, dtype=np.uint64)
    return chars.astype(np.uint8), off
