/*
 * CPU oracle for the match-count model -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load this file's library.  It shares no
 * code with the GPU library and includes none of its headers.
 *
 * What it computes (Section 2.1, Definition 2.1 "match-count model"):
 *   an object O is one value per dimension; a query Q is a list of items
 *   (dim, lo, hi), each item being the set of keywords (dim, v) with
 *   lo <= v <= hi (Example 2.1, relational ranges, inclusive).  C(r, O) is the
 *   number of elements of O inside item r, and MC(Q, O) = sum over items.
 *   The answer is the k objects of largest MC, ties broken by smaller id
 *   (the paper breaks ties randomly; the fixed total order is this
 *   implementation's reading so that results are unique).
 *
 * How (Section 3.2, "Inverted index and query processing"; the CPU-Idx
 * baseline of Section 6.1.2): keyword = (dim, value) encoded as dim*V+value,
 * a CSR "List Array" of postings (object ids, ascending) with a "Position
 * Map" of list boundaries; a query scans the lists of every keyword inside
 * each item and adds one to a per-object count array; the top k are then
 * selected from the count array.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_INVARIANT (-3)

/*
 * Build the inverted index (Section 2.1 keyword encoding; Section 3.2 List
 * Array + Position Map).  values[o*d + j] in [0, V).  off has d*V+1 entries;
 * post has n*d entries.  Keyword j*V+v holds post[off[j*V+v] .. off[j*V+v+1])
 * = ids of the objects whose value on dim j is v, in ascending id order.
 */
int oracle_build_csr(const uint32_t *values, uint64_t n, uint32_t d, uint32_t V,
                     uint64_t *off, uint32_t *post)
{
    uint64_t nkeys = (uint64_t)d * V;
    uint64_t o, key;
    uint32_t j;
    uint64_t *fill;

    if (d == 0 || V == 0)
        return ORACLE_EINVAL;
    memset(off, 0, sizeof(uint64_t) * (nkeys + 1));
    for (o = 0; o < n; o++)
        for (j = 0; j < d; j++) {
            uint32_t v = values[o * d + j];
            if (v >= V)
                return ORACLE_EINVAL;
            off[(uint64_t)j * V + v + 1] += 1;
        }
    for (key = 0; key < nkeys; key++)
        off[key + 1] += off[key];
    fill = (uint64_t *)malloc(sizeof(uint64_t) * (nkeys ? nkeys : 1));
    if (!fill)
        return ORACLE_ENOMEM;
    memcpy(fill, off, sizeof(uint64_t) * nkeys);
    /* objects visited in ascending id order -> each list ascending */
    for (o = 0; o < n; o++)
        for (j = 0; j < d; j++) {
            key = (uint64_t)j * V + values[o * d + j];
            post[fill[key]++] = (uint32_t)o;
        }
    free(fill);
    return ORACLE_OK;
}

typedef struct {
    uint32_t count;
    uint32_t id;
} pair_t;

/* total order of the answer: count descending, then id ascending */
static int cmp_pair(const void *a, const void *b)
{
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (x->count != y->count)
        return x->count > y->count ? -1 : 1;
    if (x->id != y->id)
        return x->id < y->id ? -1 : 1;
    return 0;
}

/*
 * Answer queries q_begin .. q_end-1 with the index built above.
 *
 * items: 3 uint32 per item (dim, lo, hi); query q owns items
 *        q_off[q] .. q_off[q+1]-1.  An item is the value range lo..hi
 *        inclusive; values beyond V-1 do not exist, so hi is capped at V-1 and
 *        lo > hi is an empty item.  dim >= d is an error.
 * out_ids/out_counts: k slots per query.  Row q lists min(k, n) objects in
 *        (count desc, id asc) over all n objects (zero counts included); slots
 *        past n hold (UINT32_MAX, 0).
 * out_kth: the count of the k-th object (0 when n < k).
 * out_scanned: number of postings scanned for the query.
 *
 * Checked on every query (Definition 2.1): the counts sum to the number of
 * postings scanned, and no count exceeds the number of items.
 */
int oracle_search_idx(const uint64_t *off, const uint32_t *post, uint64_t n,
                      uint32_t d, uint32_t V, const uint64_t *q_off,
                      const uint32_t *items, uint32_t q_begin, uint32_t q_end,
                      uint32_t k, uint32_t *out_ids, uint32_t *out_counts,
                      uint32_t *out_kth, uint64_t *out_scanned)
{
    uint32_t *cnt;
    uint64_t *hist;
    pair_t *above;
    uint32_t q;
    int rc = ORACLE_OK;

    if (k == 0 || d == 0 || V == 0)
        return ORACLE_EINVAL;
    cnt = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    above = (pair_t *)malloc(sizeof(pair_t) * (k + 1));
    if (!cnt || !above) {
        free(cnt);
        free(above);
        return ORACLE_ENOMEM;
    }
    for (q = q_begin; q < q_end; q++) {
        uint64_t i0 = q_off[q], i1 = q_off[q + 1], it, p, o;
        uint64_t s = i1 - i0, total = 0, sum = 0, ge;
        uint32_t *ids = out_ids + (uint64_t)(q - q_begin) * k;
        uint32_t *cts = out_counts + (uint64_t)(q - q_begin) * k;
        uint64_t kk = n < k ? n : k, na = 0, slot;
        int64_t t;

        memset(cnt, 0, sizeof(uint32_t) * n);
        /* scan: one increment per posting of every keyword inside every item */
        for (it = i0; it < i1; it++) {
            uint32_t dim = items[3 * it], lo = items[3 * it + 1], hi = items[3 * it + 2];
            if (dim >= d) {
                rc = ORACLE_EINVAL;
                goto done;
            }
            if (hi > V - 1)
                hi = V - 1;
            if (lo > hi)
                continue;
            for (p = off[(uint64_t)dim * V + lo]; p < off[(uint64_t)dim * V + hi + 1]; p++) {
                cnt[post[p]] += 1;
                total += 1;
            }
        }
        /* selection: histogram of counts, threshold t = count of the k-th */
        hist = (uint64_t *)calloc(s + 1, sizeof(uint64_t));
        if (!hist) {
            rc = ORACLE_ENOMEM;
            goto done;
        }
        for (o = 0; o < n; o++) {
            if (cnt[o] > s) {
                free(hist);
                rc = ORACLE_INVARIANT;
                goto done;
            }
            hist[cnt[o]] += 1;
            sum += cnt[o];
        }
        if (sum != total) {
            free(hist);
            rc = ORACLE_INVARIANT;
            goto done;
        }
        t = 0;
        if (kk > 0) {
            ge = 0;
            for (t = (int64_t)s; t >= 0; t--) {
                ge += hist[t];
                if (ge >= kk)
                    break;
            }
        }
        free(hist);
        /* objects strictly above t: fewer than kk of them; sort them */
        for (o = 0; o < n && kk > 0; o++)
            if ((int64_t)cnt[o] > t) {
                above[na].count = cnt[o];
                above[na].id = (uint32_t)o;
                na++;
            }
        qsort(above, na, sizeof(pair_t), cmp_pair);
        for (slot = 0; slot < na; slot++) {
            ids[slot] = above[slot].id;
            cts[slot] = above[slot].count;
        }
        /* then objects equal to t, ascending id, until kk slots are filled */
        for (o = 0; o < n && slot < kk; o++)
            if ((int64_t)cnt[o] == t) {
                ids[slot] = (uint32_t)o;
                cts[slot] = (uint32_t)t;
                slot++;
            }
        for (; slot < k; slot++) {
            ids[slot] = UINT32_MAX;
            cts[slot] = 0;
        }
        if (out_kth)
            out_kth[q - q_begin] = (n >= k) ? (uint32_t)t : 0;
        if (out_scanned)
            out_scanned[q - q_begin] = total;
    }
done:
    free(cnt);
    free(above);
    return rc;
}

/*
 * Full count vector of one query (Definition 2.1), by the same index scan.
 * out_counts has n entries.  Returns the number of postings scanned in
 * *out_scanned.
 */
int oracle_match_counts(const uint64_t *off, const uint32_t *post, uint64_t n,
                        uint32_t d, uint32_t V, const uint32_t *items,
                        uint64_t n_items, uint32_t *out_counts,
                        uint64_t *out_scanned)
{
    uint64_t it, p, total = 0;
    memset(out_counts, 0, sizeof(uint32_t) * n);
    for (it = 0; it < n_items; it++) {
        uint32_t dim = items[3 * it], lo = items[3 * it + 1], hi = items[3 * it + 2];
        if (dim >= d)
            return ORACLE_EINVAL;
        if (hi > V - 1)
            hi = V - 1;
        if (lo > hi)
            continue;
        for (p = off[(uint64_t)dim * V + lo]; p < off[(uint64_t)dim * V + hi + 1]; p++) {
            out_counts[post[p]] += 1;
            total += 1;
        }
    }
    if (out_scanned)
        *out_scanned = total;
    return ORACLE_OK;
}
