"""GPU parity: libgenie through its C-ABI against the CPU oracle.

Integer results (ids, counts) must be bit-exact.  LSH signatures computed in
float32 on the GPU may differ from the float64 oracle only where a projection
lies within float32 rounding of a bucket boundary: at most 1e-4 of the
(point, function) pairs.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1603_08390_amd as genie  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(ix, queries, k, stream=None):
    off, items = genie.queries_to_device(queries.q_offsets, queries.items)
    ids, cts, ws = genie.genie_search_async(ix, off, items, k, max(1, queries.max_items()),
                                            stream=stream)
    torch.cuda.synchronize()
    return genie.as_uint32(ids), genie.as_uint32(cts), genie.workspace_stats(ws)


def _check(values, V, queries, k, ix=None, qs=None, tile_log2=16):
    own = ix is None
    if own:
        ix = genie.Index(values, V, tile_log2)
    ids, cts, st = _run(ix, queries, k)
    assert st["status"] == 0, st
    oidx = oracle.build_csr(values, V)
    if qs is None:
        o_ids, o_cts, _, scanned = oracle.search_idx(oidx, queries, k)
        assert st["postings_scanned"] == int(scanned.sum())
        rows = range(queries.n_queries)
    else:
        rows = list(qs)
        o_ids = np.zeros((len(rows), k), np.uint32)
        o_cts = np.zeros((len(rows), k), np.uint32)
        for r, q in enumerate(rows):
            a, b, _, _ = oracle.search_idx(oidx, queries, k, q, q + 1)
            o_ids[r], o_cts[r] = a[0], b[0]
        ids, cts = ids[rows], cts[rows]
    bad = np.nonzero((ids != o_ids).any(axis=1) | (cts != o_cts).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} rows differ, first query {list(rows)[bad[0]]}"
    if own:
        ix.free()
    return st


def oracle_rows(values, V, queries, k, threads=16, chunk=16):
    """The oracle's answers to every query, chunks of queries on host threads
    (its C search releases the interpreter lock); returns ids, counts and the
    postings scanned per query."""
    import concurrent.futures as cf
    idx = oracle.build_csr(values, V)
    nq = queries.n_queries
    ids = np.zeros((nq, k), np.uint32)
    cts = np.zeros((nq, k), np.uint32)
    scanned = np.zeros(nq, np.uint64)

    def run(q0):
        q1 = min(nq, q0 + chunk)
        ids[q0:q1], cts[q0:q1], _, scanned[q0:q1] = oracle.search_idx(idx, queries, k, q0, q1)

    with cf.ThreadPoolExecutor(threads) as pool:
        list(pool.map(run, range(0, nq, chunk)))
    return ids, cts, scanned


def test_tiny_workload_full():
    inst = workloads.tiny()
    print("tiny", inst.n, inst.d, inst.queries.n_queries, flush=True)
    _check(inst.values, inst.V, inst.queries, inst.k)


@pytest.mark.parametrize("schedule", [1, 0])
@pytest.mark.parametrize("k", [1, 7, 100, 1000])
def test_relational_several_tiles_ragged(k, schedule):
    # 3 full tiles and a ragged fourth one; persistent workgroups and one
    # workgroup per pair
    inst = workloads.relational(n=3 * 65536 + 1234, d=8, V=32, nq=48, k=k)
    print("relational scaled", inst.n, inst.d, k, "schedule", schedule, flush=True)
    ix = genie.Index(inst.values, inst.V)
    genie.genie_index_set_scan_schedule(ix, schedule)
    _check(inst.values, inst.V, inst.queries, k, ix=ix)
    ix.free()


@pytest.mark.parametrize("schedule", [1, 0])
def test_short_runs_cursor_jumps_past_many_runs(schedule):
    """Streams with short runs on average: the run cursor finds its run from
    the ends of the next 64 runs at once, and moves on by 63 runs when none
    of them holds the position.  Most of the 500 items of a query name values
    no object holds (empty runs); about one in 70 names some of the 8 values
    every object holds, so consecutive non-empty runs lie more than 64 runs
    apart.  Two tiles, the second ragged; plain and gated (the gate set too
    high, so the exact fallback answers every query) searches."""
    rng = np.random.default_rng(20261203)
    n, d, V, nq, s, k = 70_000, 4, 512, 40, 500, 50
    values = rng.integers(0, 8, size=(n, d), dtype=np.uint32)
    items = np.zeros((nq * s, 3), np.uint32)
    for q in range(nq):
        for i in range(s):
            row = items[q * s + i]
            row[0] = i % d
            if (i + q) % 70 == 0:
                row[1] = rng.integers(0, 8)
                row[2] = row[1] + rng.integers(0, 3)
            else:
                row[1] = row[2] = rng.integers(100, 500)
    queries = workloads.Queries(np.arange(0, nq * s + 1, s, dtype=np.uint64), items)
    print("short runs, cursor jumps; schedule", schedule, flush=True)
    ix = genie.Index(values, V)
    genie.genie_index_set_scan_schedule(ix, schedule)
    _check(values, V, queries, k, ix=ix)
    oidx = oracle.build_csr(values, V)
    o_ids, o_cts, _, _ = oracle.search_idx(oidx, queries, k)
    off, d_items = genie.queries_to_device(queries.q_offsets, queries.items)
    high = torch.full((nq,), 1e9, dtype=torch.float32, device="cuda")
    g_ids, g_cts, ws = genie.genie_search_gated_async(ix, off, d_items, k, s, high, 0.0)
    torch.cuda.synchronize()
    st = genie.workspace_stats(ws)
    assert st["status"] == 0 and st["fallback_queries"] == nq, st
    assert np.array_equal(genie.as_uint32(g_ids), o_ids)
    assert np.array_equal(genie.as_uint32(g_cts), o_cts)
    ix.free()


def test_uneven_items_scaled():
    inst = workloads.uneven(n=140_000, d=16, V=64, nq=40, smin=1, smax=200)
    print("uneven scaled", inst.n, inst.queries.max_items(), flush=True)
    _check(inst.values, inst.V, inst.queries, 100)


def test_adversarial_small():
    rng = np.random.default_rng(2024)
    for trial in range(12):
        n = int(rng.integers(1, 3000))
        d = int(rng.integers(1, 6))
        V = int(rng.integers(1, 12))
        inst = workloads.random_small(rng, n, d, V, 20, 12)
        for k in (1, 5, max(1, n - 1), n, n + 3):
            if k > genie.GENIE_MAX_K:
                continue
            _check(inst.values, V, inst.queries, k)


def test_edge_cases():
    # n < k with padding, n = 1, empty queries, all-empty items
    values = np.array([[0, 1], [1, 1], [0, 0]], dtype=np.uint32)
    q = workloads.Queries(np.array([0, 0, 2, 4], np.uint64),
                          np.array([[0, 0, 0], [1, 1, 1], [0, 5, 2], [1, 3, 9]], np.uint32))
    _check(values, 2, q, 10)
    _check(values[:1], 2, q, 1)
    # every object identical: ties across tiles resolved by id
    same = np.full((140_000, 3), 2, dtype=np.uint32)
    q2 = workloads.Queries(np.array([0, 3], np.uint64),
                           np.array([[0, 2, 2], [1, 0, 3], [2, 3, 3]], np.uint32))
    _check(same, 4, q2, 100)


# Tiles of 2^15 - 1 objects: the same answers with every counter width
# (4-bit: <= 14 items, 8-bit: <= 254, 16-bit: more), ragged last tiles and
# ties across tiles.
@pytest.mark.parametrize("case", ["bits4", "bits8", "bits16", "ties"])
def test_smaller_tiles(case):
    print("tile_log2 15", case, flush=True)
    if case == "bits4":
        inst = workloads.relational(n=4 * 32767 + 5, d=12, V=16, nq=30, k=10)
        _check(inst.values, inst.V, inst.queries, 10, tile_log2=15)
    elif case == "bits8":
        inst = workloads.relational(n=5 * 32767 + 321, d=24, V=40, nq=40, k=100)
        _check(inst.values, inst.V, inst.queries, 100, tile_log2=15)
    elif case == "bits16":
        inst = workloads.uneven(n=100_000, d=16, V=64, nq=24, smin=200, smax=400)
        _check(inst.values, inst.V, inst.queries, 100, tile_log2=15)
    else:
        same = np.full((3 * 32767 + 9, 3), 2, dtype=np.uint32)
        q2 = workloads.Queries(np.array([0, 3], np.uint64),
                               np.array([[0, 2, 2], [1, 0, 3], [2, 3, 3]], np.uint32))
        _check(same, 4, q2, 1000, tile_log2=15)


# Persistent workgroups over the pair queue: the same answers for the plain
# search (several tiles, ragged), every query falling back in the gated
# search (a second persistent pass), and the count dump.
@pytest.mark.parametrize("tile_log2", [16, 15])
def test_persistent_schedule(tile_log2):
    print("persistent schedule, tile_log2", tile_log2, flush=True)
    inst = workloads.relational(n=3 * 65535 + 4321, d=20, V=40, nq=70, k=50)
    oidx = oracle.build_csr(inst.values, inst.V)
    o_ids, o_cts, kth, _ = oracle.search_idx(oidx, inst.queries, 50)
    for nt, u in ((1024, 4), (512, 8)):
        ix = genie.Index(inst.values, inst.V, tile_log2)
        genie.genie_index_set_scan_shape(ix, nt, u)
        genie.genie_index_set_scan_schedule(ix, 1)
        assert ix.info.scan_persistent == 1
        _check(inst.values, inst.V, inst.queries, 50, ix=ix)
        off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
        high = torch.full((inst.queries.n_queries,), 1e9, dtype=torch.float32, device="cuda")
        g_ids, g_cts, ws = genie.genie_search_gated_async(ix, off, items, 50,
                                                          inst.queries.max_items(), high, 0.0)
        torch.cuda.synchronize()
        st = genie.workspace_stats(ws)
        assert st["status"] == 0 and st["fallback_queries"] == inst.queries.n_queries
        assert np.array_equal(genie.as_uint32(g_ids), o_ids)
        assert np.array_equal(genie.as_uint32(g_cts), o_cts)
        counts, _ = genie.genie_match_count_async(ix, off, items, inst.queries.max_items())
        torch.cuda.synchronize()
        got = genie.as_uint32(counts)
        for q in (0, 33, 69):
            want, _ = oracle.match_counts(oidx, inst.queries.items_of(q))
            assert np.array_equal(got[q], want), q
        ix.free()


@pytest.mark.parametrize("tile_log2", [16, 15])
def test_match_count_dump_equals_oracle(tile_log2):
    inst = workloads.relational(n=2 * 65536 + 77, d=12, V=48, nq=6)
    ix = genie.Index(inst.values, inst.V, tile_log2)
    assert ix.info.tile_objects == (1 << tile_log2) - 1
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    counts, ws = genie.genie_match_count_async(ix, off, items, inst.queries.max_items())
    torch.cuda.synchronize()
    got = genie.as_uint32(counts)
    oidx = oracle.build_csr(inst.values, inst.V)
    total = 0
    for q in range(6):
        want, scanned = oracle.match_counts(oidx, inst.queries.items_of(q))
        assert np.array_equal(got[q], want), q
        # posting-sum invariant of Definition 2.1
        assert int(got[q].astype(np.int64).sum()) == scanned
        total += scanned
    assert genie.workspace_stats(ws)["postings_scanned"] == total
    ix.free()


def test_repeatable_and_stream_independent():
    inst = workloads.relational(n=100_000, d=16, V=64, nq=64)
    ix = genie.Index(inst.values, inst.V)
    a = _run(ix, inst.queries, 100)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = _run(ix, inst.queries, 100, stream=s)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ix.free()


def test_sync_host_entry_point_and_errors():
    inst = workloads.tiny(n=5000, nq=8)
    ix = genie.Index(inst.values, inst.V)
    ids, cts = genie.genie_search(ix, inst.queries.q_offsets, inst.queries.items, inst.k)
    o_ids, o_cts, _, _ = oracle.search_idx(oracle.build_csr(inst.values, inst.V), inst.queries,
                                           inst.k)
    assert np.array_equal(ids, o_ids) and np.array_equal(cts, o_cts)
    bad = inst.queries.items.copy()
    bad[3, 0] = inst.d
    with pytest.raises(genie.GenieError) as e:
        genie.genie_search(ix, inst.queries.q_offsets, bad, inst.k)
    assert e.value.code == genie.GENIE_EINVAL
    with pytest.raises(genie.GenieError) as e:
        genie.genie_search(ix, inst.queries.q_offsets, inst.queries.items, 0)
    assert e.value.code == genie.GENIE_EINVAL
    big = workloads.Queries(np.array([0, 1100], np.uint64),
                            np.zeros((1100, 3), np.uint32))
    with pytest.raises(genie.GenieError) as e:
        genie.genie_search(ix, big.q_offsets, big.items, 5)
    assert e.value.code == genie.GENIE_ERANGE
    # async: a bad dim is flagged on the device and acts as an empty item
    off, items = genie.queries_to_device(inst.queries.q_offsets, bad)
    _, _, ws = genie.genie_search_async(ix, off, items, inst.k, 16)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] & genie.STATUS_BAD_DIM
    # async: a query above max_items is flagged, not miscounted
    _, _, ws = genie.genie_search_async(ix, off, items, inst.k, 8)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] & genie.STATUS_TOO_MANY_ITEMS
    ix.free()


def test_relational_full_size_every_row():
    """1,000,000 x 32, Zipf(1.1) over 256 buckets, 1,024 queries, k = 100: the
    whole batch in one call (the benchmark's launch: tiles of 65,535 objects,
    1024 x 4, persistent workgroups), every row against the oracle, and the
    same batch with one workgroup per pair."""
    inst = workloads.relational()
    print("relational full", inst.n, inst.d, inst.queries.n_queries, flush=True)
    ix = genie.Index(inst.values, inst.V)
    assert ix.info.scan_shape == (1024, 4) and ix.info.scan_persistent == 2
    ids, cts, st = _run(ix, inst.queries, inst.k)
    assert st["status"] == 0, st
    o_ids, o_cts, scanned = oracle_rows(inst.values, inst.V, inst.queries, inst.k)
    assert st["postings_scanned"] == int(scanned.sum())
    bad = np.nonzero((ids != o_ids).any(axis=1) | (cts != o_cts).any(axis=1))[0]
    assert len(bad) == 0, f"{len(bad)} of 1024 rows differ, first {bad[0]}"
    print("stats", st, flush=True)
    genie.genie_index_set_scan_schedule(ix, 0)
    ids, cts, st = _run(ix, inst.queries, inst.k)
    assert st["status"] == 0 and st["postings_scanned"] == int(scanned.sum())
    assert np.array_equal(ids, o_ids) and np.array_equal(cts, o_cts)
    ix.free()


def test_merge_capped_histogram_bin():
    """The merge's count histogram spans 255 counts above the largest tile
    k-th count and pools larger counts in its top bin.  Four tiles, each with
    25 objects matching all 400 items of the query (count 400) and every
    other object matching none (tile k-th count 0), k = 100: the global k-th
    count (400) lies far past the top bin."""
    n = 4 * 65535
    values = np.zeros((n, 4), np.uint32)
    rng = np.random.default_rng(77)
    special = np.concatenate([t * 65535 + rng.choice(65535, 25, replace=False)
                              for t in range(4)])
    values[special] = 1
    # 40 more objects per tile hold value 1 on dim 0 only: count 100 in the
    # first query; in the second (400 items on dim 0) they tie at 400 with
    # the 100 above, and the 100 smallest of the 260 ids win
    mid = np.concatenate([t * 65535 + rng.choice(np.setdiff1d(np.arange(65535),
                                                              special % 65535), 40,
                                                 replace=False) for t in range(4)])
    values[mid, 0] = 1
    items = np.array([[j % 4, 1, 1] for j in range(400)], np.uint32)
    dim0 = np.array([[0, 1, 1]] * 400, np.uint32)
    q = workloads.Queries(np.array([0, 400, 800], np.uint64), np.concatenate([items, dim0]))
    print("capped merge bin:", n, "objects, 400 items, k = 100", flush=True)
    _check(values, 2, q, 100)
def test_lsh_signatures_vs_float64():
    inp = workloads.ann(n=100_000, nq=16)
    P = torch.from_numpy(inp.points).cuda()
    A = torch.from_numpy(inp.a).cuda()
    B = torch.from_numpy(inp.b).cuda()
    R = torch.from_numpy(inp.rehash.view(np.int64)).cuda()
    sig = genie.genie_lsh_signatures(P, A, B, inp.w, R, inp.log2_buckets)
    torch.cuda.synchronize()
    got = genie.as_uint32(sig)
    want = oracle.lsh_signatures(inp.points, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    rate = float((got != want).mean())
    print("lsh mismatch rate", rate, flush=True)
    assert rate <= 1e-4
    # batch invariance: a sub-batch gives the same rows
    sub = genie.genie_lsh_signatures(P[777:1999].contiguous(), A, B, inp.w, R, inp.log2_buckets)
    torch.cuda.synchronize()
    assert np.array_equal(genie.as_uint32(sub), got[777:1999])


def test_ann_search_on_shared_signatures():
    """tau-ANN through LSH (Section 4.1): oracle float64 signatures feed both
    sides; the match count search is then exact."""
    inp = workloads.ann(n=150_000, nq=48)
    sig = oracle.lsh_signatures(inp.points, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    qsig = oracle.lsh_signatures(inp.queries, inp.a, inp.b, inp.w, inp.rehash, inp.log2_buckets)
    q = workloads.queries_exact(qsig)
    _check(sig, 1 << inp.log2_buckets, q, inp.k)


# GEN-SPQ ablation (no Gate, no Hash Table; the k-th count by bisection over
# the exact counters): the same answers at every counter width, both tilings
# and k > n.
@pytest.mark.parametrize("case", ["relational", "uneven", "tiles15", "small"])
def test_gen_spq_ablation_equals_oracle(case):
    print("gen-spq", case, flush=True)
    if case == "relational":
        inst = workloads.relational(n=3 * 65535 + 77, d=20, V=40, nq=40, k=100)
        lg, k = 16, 100
    elif case == "uneven":
        inst = workloads.uneven(n=100_000, d=16, V=64, nq=16, smin=100, smax=400)
        lg, k = 16, 100
    elif case == "tiles15":
        inst = workloads.relational(n=4 * 32767 + 5, d=12, V=16, nq=30, k=10)
        lg, k = 15, 10
    else:
        inst = workloads.relational(n=900, d=6, V=10, nq=8, k=1000)
        lg, k = 16, 1000
    ix = genie.Index(inst.values, inst.V, lg)
    off, items = genie.queries_to_device(inst.queries.q_offsets, inst.queries.items)
    ids, cts, ws = genie.genie_search_spq_async(ix, off, items, k, inst.queries.max_items())
    torch.cuda.synchronize()
    o_ids, o_cts, _, scanned = oracle.search_idx(oracle.build_csr(inst.values, inst.V),
                                                 inst.queries, k)
    st = genie.workspace_stats(ws)
    assert st["status"] == 0 and st["gate_passes"] == 0 and st["ht_inserts"] == 0
    assert st["postings_scanned"] == int(scanned.sum())
    assert np.array_equal(genie.as_uint32(ids), o_ids)
    assert np.array_equal(genie.as_uint32(cts), o_cts)
    ix.free()


@pytest.mark.parametrize("schedule", [1, 0])
def test_compact_position_map(schedule):
    """An index with many keywords per posting (4,096 buckets on 8 dims over
    3 tiles and a ragged fourth) keeps its Position Map in the compact form
    (checkpoints every 8 keywords plus uint16 run lengths); range items of up
    to 41 keywords cross the 8-keyword groups.  Plain and gated answers
    against the oracle."""
    rng = np.random.default_rng(808)
    n, d, V = 3 * 65535 + 999, 8, 4096
    values = rng.integers(0, V, size=(n, d), dtype=np.uint32)
    qs = workloads.queries_random_width(rng, values, V, 40, wmax=40)
    ix = genie.Index(values, V)
    assert ix.info.map_compact == 1
    assert ix.info.map_bytes < ix.info.n_tiles * (d * V + 1) * 8 / 2
    genie.genie_index_set_scan_schedule(ix, schedule)
    print("compact map: schedule", schedule, ix.info, flush=True)
    _check(values, V, qs, 100, ix=ix)
    o_ids, o_cts, o_kth, _ = oracle.search_idx(oracle.build_csr(values, V), qs, 100)
    off, items = genie.queries_to_device(qs.q_offsets, qs.items)
    pred = torch.from_numpy(o_kth.astype(np.float32)).cuda()
    g_ids, g_cts, ws = genie.genie_search_gated_async(ix, off, items, 100, qs.max_items(), pred,
                                                      0.0)
    torch.cuda.synchronize()
    assert genie.workspace_stats(ws)["status"] == 0
    assert np.array_equal(genie.as_uint32(g_ids), o_ids)
    assert np.array_equal(genie.as_uint32(g_cts), o_cts)
    ix.free()
