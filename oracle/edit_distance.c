/*
 * Edit distance for the sequence-search oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * The distance of Section 5.1 (sequence similarity under edit distance):
 * the least number of single-character insertions, deletions and
 * substitutions that turn a into b (Levenshtein distance).  Computed by the
 * textbook dynamic programme (Wagner and Fischer): D[i][j] is the distance
 * of the prefixes a[0..i) and b[0..j),
 *   D[i][0] = i, D[0][j] = j,
 *   D[i][j] = min(D[i-1][j] + 1,                      delete a[i-1]
 *                 D[i][j-1] + 1,                      insert b[j-1]
 *                 D[i-1][j-1] + (a[i-1] != b[j-1]))   match or substitute
 * kept one row at a time.  Plain, slow, obviously correct; it shares no code
 * with the GPU library.
 */
#include <stdint.h>
#include <stdlib.h>

uint32_t oracle_edit_distance(const uint8_t *a, uint32_t la, const uint8_t *b, uint32_t lb)
{
    uint32_t *prev = (uint32_t *)malloc(((size_t)lb + 1) * sizeof(uint32_t));
    uint32_t *cur = (uint32_t *)malloc(((size_t)lb + 1) * sizeof(uint32_t));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return UINT32_MAX;
    }
    for (uint32_t j = 0; j <= lb; j++)
        prev[j] = j;
    for (uint32_t i = 1; i <= la; i++) {
        cur[0] = i;
        for (uint32_t j = 1; j <= lb; j++) {
            uint32_t del = prev[j] + 1;
            uint32_t ins = cur[j - 1] + 1;
            uint32_t sub = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1u : 0u);
            uint32_t m = del < ins ? del : ins;
            cur[j] = m < sub ? m : sub;
        }
        uint32_t *t = prev;
        prev = cur;
        cur = t;
    }
    uint32_t d = prev[lb];
    free(prev);
    free(cur);
    return d;
}

/*
 * Many pairs: pair p is (a_chars[a_off[ai[p]] .. a_off[ai[p]+1]),
 * b_chars[b_off[bi[p]] .. b_off[bi[p]+1])); out[p] = their distance.
 * Returns 0, or -1 if an allocation failed.
 */
int oracle_edit_distances(const uint8_t *a_chars, const uint64_t *a_off, const uint64_t *ai,
                          const uint8_t *b_chars, const uint64_t *b_off, const uint64_t *bi,
                          uint64_t n_pairs, uint32_t *out)
{
    for (uint64_t p = 0; p < n_pairs; p++) {
        const uint64_t a0 = a_off[ai[p]], a1 = a_off[ai[p] + 1];
        const uint64_t b0 = b_off[bi[p]], b1 = b_off[bi[p] + 1];
        out[p] = oracle_edit_distance(a_chars + a0, (uint32_t)(a1 - a0), b_chars + b0,
                                      (uint32_t)(b1 - b0));
        if (out[p] == UINT32_MAX)
            return -1;
    }
    return 0;
}
