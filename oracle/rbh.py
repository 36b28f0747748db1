"""CPU oracle for random binning hashing (RBH) of the Laplacian kernel and its
MurmurHash3 re-hash (Section 4.1.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``murmur3_32_words`` -- MurmurHash3, x86 32-bit variant, written from its
  public description (Appleby's SMHasher), for keys made of whole 4-byte
  little-endian blocks: per block k: k *= c1, k = rotl(k, 15), k *= c2,
  h ^= k, h = rotl(h, 13), h = 5 h + 0xe6546b64; then h ^= length in bytes
  and the final avalanche (fmix32).
* ``rbh_bins_f64`` -- one RBH function per row of (g, u): a randomly shifted
  regular grid with pitch g_j and shift u_j on every dimension; the bin of
  point p is floor((p_j - u_j) / g_j) per dimension, computed in float64.
  Reading: the paper names one cell size g sampled from p(s) = s k''(s) and
  states that the collision probability equals the kernel; for the
  Laplacian kernel exp(-||p - q||_1 / sigma) that holds when every dimension
  draws its own pitch g_j from the Gamma(2, sigma) density (s / sigma^2)
  e^(-s / sigma) and its shift u_j uniformly from [0, g_j), which is the
  construction used here.
* ``rbh_signatures`` -- bins of every function, re-hashed: bucket =
  MurmurHash3(bins as int32 blocks, seed_i) >> (32 - log2 D).
* ``exact_knn_l1`` -- exact L1 neighbours (the Laplacian kernel is monotone
  in the L1 distance).
"""
from __future__ import annotations

import numpy as np

C1 = np.uint32(0xCC9E2D51)
C2 = np.uint32(0x1B873593)
M32 = 0xFFFFFFFF


def _rotl(x: np.ndarray, r: int) -> np.ndarray:
    return (x << np.uint32(r)) | (x >> np.uint32(32 - r))


def _fmix32(h: np.ndarray) -> np.ndarray:
    h = h ^ (h >> np.uint32(16))
    h = h * np.uint32(0x85EBCA6B)
    h = h ^ (h >> np.uint32(13))
    h = h * np.uint32(0xC2B2AE35)
    h = h ^ (h >> np.uint32(16))
    return h


def murmur3_32_words(words: np.ndarray, seed) -> np.ndarray:
    """MurmurHash3_x86_32 of each row of `words` (uint32 [n, L], L >= 1, the
    little-endian 4-byte blocks of a 4L-byte key) with per-row or shared
    seed; returns uint32 [n]."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.ndim == 1:
        w = w[None, :]
    n, L = w.shape
    with np.errstate(over="ignore"):
        h = np.broadcast_to(np.asarray(seed, dtype=np.uint32), (n,)).copy()
        for j in range(L):
            k = w[:, j] * C1
            k = _rotl(k, 15)
            k = k * C2
            h = h ^ k
            h = _rotl(h, 13)
            h = h * np.uint32(5) + np.uint32(0xE6546B64)
        h = h ^ np.uint32((4 * L) & M32)
        return _fmix32(h)


def rbh_bins_f64(points: np.ndarray, g: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Bins of every point under every function: int64 [n, m, d]."""
    p = np.asarray(points, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    return np.floor((p[:, None, :] - u[None, :, :]) / g[None, :, :]).astype(np.int64)


def rbh_signatures(points: np.ndarray, g: np.ndarray, u: np.ndarray, seeds: np.ndarray,
                   log2_buckets: int, chunk: int = 4096) -> np.ndarray:
    """uint32 [n, m] buckets: MurmurHash3 of the function's bin vector (as
    int32 blocks), seeded per function, top log2_buckets bits."""
    n = points.shape[0]
    m = g.shape[0]
    out = np.empty((n, m), dtype=np.uint32)
    seeds = np.asarray(seeds, dtype=np.uint32)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        bins = rbh_bins_f64(points[r0:r1], g, u)                   # [c, m, d]
        words = bins.astype(np.int32).view(np.uint32)                # two's complement blocks
        for i in range(m):
            h = murmur3_32_words(words[:, i, :], seeds[i])
            out[r0:r1, i] = h >> np.uint32(32 - log2_buckets)
    return out


def laplacian_kernel(p: np.ndarray, q: np.ndarray, sigma: float) -> np.ndarray:
    return np.exp(-np.abs(np.asarray(p, np.float64) - np.asarray(q, np.float64)).sum(-1) / sigma)


def exact_knn_l1(points: np.ndarray, queries: np.ndarray, k: int, chunk: int = 65536):
    """Exact L1 k nearest neighbours in float64, ordered by (distance, id)."""
    P = np.asarray(points, dtype=np.float64)
    ids = np.zeros((len(queries), k), dtype=np.int64)
    dist = np.zeros((len(queries), k), dtype=np.float64)
    for qi, q in enumerate(np.asarray(queries, dtype=np.float64)):
        d = np.concatenate([np.abs(P[c:c + chunk] - q).sum(1) for c in range(0, len(P), chunk)])
        order = np.lexsort((np.arange(len(P)), d))[:k]
        ids[qi], dist[qi] = order, d[order]
    return ids, dist
