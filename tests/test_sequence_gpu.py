"""Sequence search under edit distance (Section 5.1) on the GPU against the
oracle: the keyword-set index, query decomposition into ordered n-grams
(checked through the top-K candidates and full count vectors, bit-exact),
Algorithm 2's answer and Theorem 5.2's certificate (exact), on title-like
text over several tiles with a ragged tail, small alphabets with many
repeated n-grams, empty, short, out-of-alphabet and maximum-length queries,
K >= n, and k = K = GENIE_MAX_K."""
import numpy as np
import pytest

import workloads
from oracle import UINT32_MAX
from oracle import sequence as osq

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev_q(qc, qo):
    qc = np.ascontiguousarray(qc, dtype=np.uint8)
    d_qc = torch.from_numpy(qc if qc.size else np.zeros(1, np.uint8)).cuda()[:qc.size]
    d_qo = torch.from_numpy(np.ascontiguousarray(qo, dtype=np.uint64).view(np.int64)).cuda()
    return d_qc, d_qo


def _extra_queries(rng, chars, off):
    """Edge cases appended to a batch: empty, shorter than the n-gram, bytes
    outside the data alphabet, one n-gram repeated, an exact data sequence,
    and a long query of several 64-bit words."""
    s5 = chars[int(off[5]):int(off[6])].tobytes()
    long_q = chars[int(off[0]):int(off[0]) + 200].tobytes()
    return [b"", b"a", b"ab", b"ZZ##", b"e" * 60, s5, long_q,
            b"q" + s5[1:] + b"\x00\xff"]


def _batch(inp_chars, inp_off, qc, qo, extra):
    qs = [qc[int(qo[j]):int(qo[j + 1])].tobytes() for j in range(qo.size - 1)] + extra
    return workloads.pack_sequences(qs)


def _check_search(chars, off, qc, qo, gram, K, k, tile_log2=16, fused=True):
    print("seq", off.size - 1, "queries", qo.size - 1, "gram", gram, "K", K, "k", k,
          "tile_log2", tile_log2, flush=True)
    sx = genie.SeqIndex(chars, off, gram, tile_log2)
    corpus = osq.SeqCorpus(chars, off, gram)
    want = osq.sequence_search(corpus, qc, qo, K, k)
    d_qc, d_qo = _dev_q(qc, qo)
    max_qlen = int(np.diff(qo).max()) if qo.size > 1 else 0
    # staged: decomposition, match-count top-K, verification
    items = genie.genie_seq_decompose_async(sx, d_qc, d_qo)
    c_ids, c_cts, ws = genie.genie_search_async(sx.match_index, d_qo, items, K, max(max_qlen, 1))
    ids, dist, cert = genie.genie_seq_verify_async(sx, d_qc, d_qo, max_qlen, c_ids, c_cts, k)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] == 0
    assert np.array_equal(genie.as_uint32(c_ids), want.cand_ids)
    assert np.array_equal(genie.as_uint32(c_cts), want.cand_counts)
    assert np.array_equal(genie.as_uint32(ids), want.ids)
    assert np.array_equal(genie.as_uint32(dist), want.dist)
    assert np.array_equal(genie.as_uint32(cert)[:qo.size - 1], want.cert)
    if fused:
        f_ids, f_dist, f_cert, ws = genie.genie_seq_search_async(sx, d_qc, d_qo, max_qlen, K, k)
        torch.cuda.synchronize()
        assert genie.workspace_stats(ws)["status"] == 0
        assert torch.equal(f_ids, ids) and torch.equal(f_dist, dist)
        assert torch.equal(f_cert[:qo.size - 1], cert[:qo.size - 1])
    sx.free()
    return want


def test_keyword_sets_index_equals_the_dense_index():
    inst = workloads.relational(n=70_000, d=8, V=32, nq=30, k=20)
    n, d = inst.values.shape
    keys = (np.arange(d, dtype=np.uint32)[None, :] * inst.V + inst.values).reshape(-1)
    obj_off = np.arange(n + 1, dtype=np.uint64) * d
    sets = genie.genie_build_index_sets(obj_off, keys, d * inst.V, 15)
    dense = genie.Index(inst.values, inst.V, 15)
    # one-keyword items on both: (dim, v, v) on the dense index is the key dim*V+v
    rng = np.random.default_rng(2)
    q_items, q_off = [], [0]
    for _ in range(30):
        s = int(rng.integers(0, 20))
        dims = rng.integers(0, d, size=s)
        vals = rng.integers(0, inst.V, size=s)
        q_items += [(int(a), int(v), int(v)) for a, v in zip(dims, vals)]
        q_off.append(len(q_items))
    dense_items = np.array(q_items, dtype=np.uint32).reshape(-1, 3)
    set_items = np.stack([np.zeros(len(q_items)), dense_items[:, 0] * inst.V + dense_items[:, 1],
                          dense_items[:, 0] * inst.V + dense_items[:, 2]], 1).astype(np.uint32)
    off = np.array(q_off, dtype=np.uint64)
    d_off, d_di = genie.queries_to_device(off, dense_items)
    _, d_si = genie.queries_to_device(off, set_items)
    a_ids, a_cts, _ = genie.genie_search_async(dense, d_off, d_di, 20, 20)
    b_ids, b_cts, ws = genie.genie_search_async(sets, d_off, d_si, 20, 20)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] == 0
    assert torch.equal(a_ids, b_ids) and torch.equal(a_cts, b_cts)
    # a range item on a keyword-set index is flagged and counts nothing
    bad = set_items.copy()
    bad[0, 2] = bad[0, 1] + 3
    _, d_bad = genie.queries_to_device(off, bad)
    _, _, ws = genie.genie_search_async(sets, d_off, d_bad, 20, 20)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] & genie.STATUS_RANGE_ON_SET
    sets.free()
    dense.free()


def test_text_several_tiles_and_edge_queries():
    rng = np.random.default_rng(7)
    chars, off = workloads.text_corpus(rng, 70_000, vocab=3000)
    qc, qo, _ = workloads.modified_queries(rng, chars, off, 48, 40, 0.2)
    qc, qo = _batch(chars, off, qc, qo, _extra_queries(rng, chars, off))
    want = _check_search(chars, off, qc, qo, 3, 32, 1, tile_log2=15)
    assert 0 < want.cert.sum() < want.cert.size
    _check_search(chars, off, qc, qo, 3, 16, 3, tile_log2=16, fused=False)


def test_small_alphabet_repeated_ngrams_and_all_candidates():
    rng = np.random.default_rng(8)
    chars, off = workloads.random_sequences(rng, 900, b"abc", 0, 40)
    qs = [bytes(rng.choice(list(b"abc"), size=int(rng.integers(0, 45))).tolist())
          for _ in range(40)] + [b"aaaaaaaaaaaaaaaa", b"abcabcabcabc", b"d"]
    qc, qo = workloads.pack_sequences(qs)
    for gram in (2, 3, 5):
        _check_search(chars, off, qc, qo, gram, 24, 4)
    # K >= n: every sequence is a candidate; the full count vector is checked
    small_c, small_o = workloads.random_sequences(rng, 300, b"ab", 0, 30)
    want = _check_search(small_c, small_o, qc, qo, 3, 320, 5)
    corpus = osq.SeqCorpus(small_c, small_o, 3)
    for j in range(3):
        q = qc[int(qo[j]):int(qo[j + 1])].tobytes()
        mc = corpus.match_counts(q)
        ids = want.cand_ids[j][:300].astype(np.int64)
        assert np.array_equal(want.cand_counts[j][:300], mc[ids])
    assert want.cert.all()


def test_maximum_sizes():
    rng = np.random.default_rng(9)
    chars, off = workloads.random_sequences(rng, 3000, b"abcdefgh", 900, 1100)
    qs = [chars[int(off[i]):int(off[i]) + genie.GENIE_MAX_ITEMS].tobytes() for i in range(4)]
    qs[1] = qs[1][:-300] + b"h" * 300
    qc, qo = workloads.pack_sequences(qs)
    # K = GENIE_MAX_K with 1,024 items per query needs the smaller tiles' LDS
    _check_search(chars, off, qc, qo, 4, genie.GENIE_MAX_K, genie.GENIE_MAX_K, tile_log2=15)
    _check_search(chars, off, qc, qo, 4, 64, 1)


def test_verify_distances_for_every_pattern_width():
    """Bit-vector widths of 1..16 words: distances equal the dynamic
    programme's on given candidates (the answer is their order by
    (distance, position)); the certificate follows Theorem 5.2."""
    rng = np.random.default_rng(10)
    chars, off = workloads.random_sequences(rng, 500, b"acgt", 0, 1100)
    sx = genie.SeqIndex(chars, off, 3)
    for qlen in (1, 63, 64, 65, 128, 129, 256, 300, 512, 700, 1024):
        nq, K, k = 6, 40, 3
        qs = [bytes(rng.choice(list(b"acgt"), size=int(rng.integers(max(0, qlen - 5), qlen + 1)))
                    .tolist()) for _ in range(nq)]
        qc, qo = workloads.pack_sequences(qs)
        cand = rng.integers(0, 500, size=(nq, K)).astype(np.uint32)
        cand[0, -5:] = UINT32_MAX                      # empty slots
        counts = np.sort(rng.integers(0, 50, size=(nq, K)), axis=1)[:, ::-1].astype(np.uint32)
        d_qc, d_qo = _dev_q(qc, qo)
        ids, dist, cert = genie.genie_seq_verify_async(
            sx, d_qc, d_qo, qlen, torch.from_numpy(cand.view(np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(counts).view(np.int32)).cuda(), k)
        torch.cuda.synchronize()
        for j in range(nq):
            valid = cand[j] != UINT32_MAX
            eds = np.full(K, UINT32_MAX, dtype=np.uint32)
            eds[valid] = osq.edit_distances(qc, qo, np.full(valid.sum(), j, np.uint64), chars,
                                            off, cand[j][valid].astype(np.uint64))
            order = sorted((int(e), p) for p, e in enumerate(eds))[:k]
            assert genie.as_uint32(dist)[j].tolist() == [e for e, _ in order], (qlen, j)
            assert genie.as_uint32(ids)[j].tolist() == [
                UINT32_MAX if e == UINT32_MAX else int(cand[j][p]) for e, p in order]
            want_cert = osq.certified(len(qs[j]), 3, cand[j], counts[j],
                                      [e for e, _ in order], k, 500)
            assert int(genie.as_uint32(cert)[j]) == int(want_cert)
    sx.free()


def test_full_size_sampled_against_oracle():
    """The benchmark's workload (5,000,000 title-like strings, 1,024 queries
    of 40 characters with 20 % replaced, 3-grams, K = 32, k = 1) in the
    benchmark's launch configuration; the oracle checks a sample of queries."""
    inp = workloads.sequence()
    print("sequence workload built", inp.n, inp.nq, flush=True)
    sx = genie.SeqIndex(inp.chars, inp.offsets, inp.gram)
    print("index built", sx.info, flush=True)
    d_qc, d_qo = _dev_q(inp.qchars, inp.qoffsets)
    ids, dist, cert, ws = genie.genie_seq_search_async(sx, d_qc, d_qo, 40, inp.K, inp.k)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] == 0
    ids, dist, cert = genie.as_uint32(ids), genie.as_uint32(dist), genie.as_uint32(cert)
    sx.free()
    corpus = osq.SeqCorpus(inp.chars, inp.offsets, inp.gram)
    print("oracle corpus ready", flush=True)
    sample = [0, 1, 517, inp.nq - 1]
    want = osq.sequence_search(corpus, inp.qchars, inp.qoffsets, inp.K, inp.k, sample)
    for r, j in enumerate(sample):
        assert ids[j].tolist() == want.ids[r].tolist()
        assert dist[j].tolist() == want.dist[r].tolist()
        assert int(cert[j]) == int(want.cert[r])
    # every query's source is a data sequence at distance at most 8 (20 % of 40)
    assert np.all(dist[:, 0] <= 8)
