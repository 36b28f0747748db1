"""Pins of the sequence-search oracle (Section 5.1) against things other than
itself: the paper's Example 5.1, hand-worked match counts, textbook and
brute-force (breadth-first search over single edits) edit distances,
Lemma 5.1 against the set definition, Theorem 5.1 on random edited pairs,
Algorithm 2 against the plain definition of its answer, and Theorem 5.2's
certificate against exhaustive search."""
import itertools
import json
import os
from collections import deque

import numpy as np
import pytest

import workloads
from oracle import UINT32_MAX
from oracle import sequence as osq

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "ordered_ngrams_example.json")))


def test_example_5_1_ordered_ngrams():
    got = osq.ordered_ngrams(GOLD["sequence"].encode(), GOLD["n"])
    assert [(g.decode(), i) for g, i in got] == [tuple(x) for x in GOLD["ordered_ngrams"]]


def test_hand_worked_counts_and_bound():
    h = GOLD["hand_worked"]
    s, n = GOLD["sequence"].encode(), GOLD["n"]
    assert osq.mc_ordered(s, h["query"].encode(), n) == h["mc"]
    assert osq.mc_by_counts(s, h["query"].encode(), n) == h["mc"]
    e = h["edited"].encode()
    assert osq.edit_distance(s, e) == h["edit_distance_edited"]
    assert osq.mc_ordered(s, e, n) == h["mc_edited"]


def test_lemma_5_1_set_definition_equals_min_counts():
    rng = np.random.default_rng(3)
    for _ in range(400):
        n = int(rng.integers(1, 5))
        a = bytes(rng.choice(list(b"ab"), size=int(rng.integers(0, 14))).tolist())
        b = bytes(rng.choice(list(b"abc"), size=int(rng.integers(0, 14))).tolist())
        assert osq.mc_ordered(a, b, n) == osq.mc_by_counts(a, b, n)
        assert osq.mc_ordered(a, b, n) == osq.mc_ordered(b, a, n)


@pytest.mark.parametrize("a,b,d", [(b"kitten", b"sitting", 3), (b"flaw", b"lawn", 2),
                                   (b"intention", b"execution", 5), (b"", b"abc", 3),
                                   (b"abc", b"", 3), (b"abc", b"abc", 0),
                                   (b"sunday", b"saturday", 3), (b"ab", b"ba", 2)])
def test_edit_distance_textbook_values(a, b, d):
    assert osq.edit_distance(a, b) == d


def _bfs_distances(src: bytes, alphabet: bytes, max_len: int):
    """Distance from src to every string over the alphabet of length <= max_len,
    by breadth-first search over single insertions, deletions, substitutions."""
    dist = {src: 0}
    dq = deque([src])
    while dq:
        s = dq.popleft()
        nxt = set()
        for i in range(len(s)):
            nxt.add(s[:i] + s[i + 1:])
            for c in alphabet:
                nxt.add(s[:i] + bytes([c]) + s[i + 1:])
        if len(s) < max_len:
            for i in range(len(s) + 1):
                for c in alphabet:
                    nxt.add(s[:i] + bytes([c]) + s[i:])
        for t in nxt:
            if t not in dist:
                dist[t] = dist[s] + 1
                dq.append(t)
    return dist


def test_edit_distance_equals_breadth_first_search():
    alphabet = b"abc"
    strings = [bytes(p) for L in range(0, 4) for p in itertools.product(alphabet, repeat=L)]
    for src in strings[::3]:
        bfs = _bfs_distances(src, alphabet, 4)
        for t in strings:
            assert osq.edit_distance(src, t) == bfs[t], (src, t)


def _random_edits(rng, s: bytes, m: int, alphabet: bytes) -> bytes:
    s = bytearray(s)
    for _ in range(m):
        op = rng.integers(0, 3)
        if op == 0 and len(s):
            del s[int(rng.integers(0, len(s)))]
        elif op == 1:
            s.insert(int(rng.integers(0, len(s) + 1)), alphabet[int(rng.integers(0, len(alphabet)))])
        elif len(s):
            s[int(rng.integers(0, len(s)))] = alphabet[int(rng.integers(0, len(alphabet)))]
    return bytes(s)


def test_theorem_5_1_count_bound_on_edited_pairs():
    rng = np.random.default_rng(11)
    tight = 0
    for _ in range(600):
        n = int(rng.integers(2, 5))
        alphabet = b"abcd"[:int(rng.integers(2, 5))]
        s = bytes(rng.choice(list(alphabet), size=int(rng.integers(0, 30))).tolist())
        q = _random_edits(rng, s, int(rng.integers(0, 6)), alphabet)
        tau = osq.edit_distance(s, q)
        mc = osq.mc_ordered(s, q, n)
        bound = max(len(q), len(s)) - n + 1 - tau * n
        assert mc >= bound, (s, q, n, tau, mc)
        tight += mc == bound
    assert tight > 0   # the bound is attained sometimes: it is not slack everywhere


def _small_corpus(seed, n=3000, nq=30, frac=0.3):
    rng = np.random.default_rng(seed)
    chars, off = workloads.text_corpus(rng, n, vocab=300)
    qc, qo, src = workloads.modified_queries(rng, chars, off, nq, 40, frac)
    return chars, off, qc, qo, src


def test_corpus_counts_equal_the_set_definition():
    rng = np.random.default_rng(4)
    chars, off = workloads.random_sequences(rng, 300, b"abc", 0, 25)
    corpus = osq.SeqCorpus(chars, off, 3)
    for q in (b"abcabcaab", b"aaaaaaa", b"", b"ab", b"cbacbacbbbaaabc"):
        mc = corpus.match_counts(q)
        want = [osq.mc_ordered(corpus.seq(i), q, 3) for i in range(corpus.N)]
        assert mc.tolist() == want


@pytest.mark.parametrize("k", [1, 2, 5])
def test_algorithm_2_answer_is_the_closest_candidates(k):
    chars, off, qc, qo, src = _small_corpus(5, frac=0.4)
    corpus = osq.SeqCorpus(chars, off, 3)
    for j in range(qo.size - 1):
        q = qc[int(qo[j]):int(qo[j + 1])].tobytes()
        ids, cts = corpus.candidates(q, 24)
        pos, dist = osq.verify(q, ids, cts, corpus.seq, 3, k)
        eds = [osq.edit_distance(q, corpus.seq(int(i))) for i in ids]
        want = sorted((e, p) for p, e in enumerate(eds))[:k]
        assert list(zip(dist, pos)) == want


def test_algorithm_2_on_small_alphabets_with_ties():
    """Count order and distance order disagree often here, and distances tie:
    an early break or a tie given to the later candidate changes the answer."""
    rng = np.random.default_rng(12)
    broke = 0
    for n in (2, 3):
        chars, off = workloads.random_sequences(rng, 400, b"abcd", 3, 22)
        corpus = osq.SeqCorpus(chars, off, n)
        for _ in range(60):
            q = bytes(rng.choice(list(b"abcd"), size=int(rng.integers(4, 20))).tolist())
            for K, k in ((8, 1), (30, 1), (30, 3)):
                ids, cts = corpus.candidates(q, K)
                pos, dist = osq.verify(q, ids, cts, corpus.seq, n, k)
                eds = [osq.edit_distance(q, corpus.seq(int(i))) for i in ids]
                want = sorted((e, p) for p, e in enumerate(eds))[:k]
                assert list(zip(dist, pos)) == want, (q, n, K, k)
                theta = len(q) - n + 1 - n * (want[-1][0] - 1)
                broke += any(int(c) < theta for c in cts)
    assert broke > 0   # the filtering bound does stop some scans


def _cluster_corpus(rng, n_base, variants, alphabet, lmin, lmax, max_edits):
    seqs = []
    for _ in range(n_base):
        base = bytes(rng.choice(list(alphabet), size=int(rng.integers(lmin, lmax + 1))).tolist())
        seqs.append(base)
        for _ in range(variants):
            seqs.append(_random_edits(rng, base, int(rng.integers(1, max_edits + 1)), alphabet))
    order = rng.permutation(len(seqs))
    return [seqs[i] for i in order]


def test_algorithm_2_on_near_duplicate_clusters():
    """Many candidates at small, tied distances with counts close to the
    filtering bound: the break, the length filter and the tie rule all
    decide answers here."""
    rng = np.random.default_rng(21)
    for n in (2, 3):
        seqs = _cluster_corpus(rng, 40, 12, b"abc", 8, 24, 4)
        chars, off = workloads.pack_sequences(seqs)
        corpus = osq.SeqCorpus(chars, off, n)
        for t in range(150):
            base = seqs[int(rng.integers(0, len(seqs)))]
            q = _random_edits(rng, base, int(rng.integers(0, 4)), b"abc")
            for K, k in ((6, 1), (20, 1), (20, 2), (40, 4)):
                ids, cts = corpus.candidates(q, K)
                pos, dist = osq.verify(q, ids, cts, corpus.seq, n, k)
                eds = [osq.edit_distance(q, corpus.seq(int(i))) for i in ids]
                want = sorted((e, p) for p, e in enumerate(eds))[:k]
                assert list(zip(dist, pos)) == want, (q, n, K, k)


def test_theorem_5_2_certificate_is_sound_and_not_vacuous():
    cert_seen = uncert_seen = 0
    for frac, K, k in ((0.1, 4, 1), (0.1, 16, 3), (0.2, 16, 1), (0.3, 16, 1)):
        chars, off, qc, qo, src = _small_corpus(6, n=4000, nq=40, frac=frac)
        corpus = osq.SeqCorpus(chars, off, 3)
        ans = osq.sequence_search(corpus, qc, qo, K, k)
        for j in range(qo.size - 1):
            q = qc[int(qo[j]):int(qo[j + 1])].tobytes()
            if ans.cert[j]:
                allq = osq.edit_distances(np.frombuffer(q, np.uint8),
                                          np.array([0, len(q)], np.uint64),
                                          np.zeros(corpus.N, np.uint64), corpus.chars,
                                          corpus.offsets, np.arange(corpus.N, dtype=np.uint64))
                assert sorted(allq.tolist())[:k] == ans.dist[j].tolist()
                cert_seen += 1
            else:
                uncert_seen += 1
    print("certified", cert_seen, "not certified", uncert_seen)
    assert cert_seen > 0 and uncert_seen > 0


def test_certificate_condition_and_all_candidate_case():
    ids = np.arange(32, dtype=np.uint32)
    cts = np.full(32, 10, dtype=np.uint32)
    # |Q| = 40, n = 3, tau = 8: bound 38 - 24 = 14
    assert osq.certified(40, 3, ids, cts, [8], 1, 10_000)
    cts[-1] = 14
    assert not osq.certified(40, 3, ids, cts, [8], 1, 10_000)
    assert osq.certified(40, 3, ids, cts, [8], 1, 32)       # every object a candidate
    ids2, cts2 = ids.copy(), cts.copy()
    ids2[20:] = UINT32_MAX
    assert osq.certified(40, 3, ids2, cts2, [8], 1, 20)


def test_search_pads_when_fewer_objects_than_answers():
    chars, off = workloads.pack_sequences([b"abcab", b"bcabc"])
    corpus = osq.SeqCorpus(chars, off, 2)
    qc, qo = workloads.pack_sequences([b"abcabc"])
    ans = osq.sequence_search(corpus, qc, qo, 4, 3)
    assert ans.cand_ids[0].tolist() == [0, 1, UINT32_MAX, UINT32_MAX]
    assert ans.ids[0].tolist() == [0, 1, UINT32_MAX]
    assert ans.dist[0].tolist() == [1, 1, UINT32_MAX]
    assert ans.cert[0] == 1
