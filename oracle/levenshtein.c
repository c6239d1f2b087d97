/*
 * Ground-truth edit distance -- TEST INFRASTRUCTURE ONLY.
 *
 * The paper labels each pair with the unit-cost global (end-to-end) edit
 * distance computed by Edlib under threshold E (Sec. 3.1; Supplementary
 * Sec. 12): a pair is similar iff its distance is <= E.  False accepts are
 * dissimilar pairs the filter accepts, false rejects are similar pairs it
 * rejects (Sec. 3.2).  Both functions below are the textbook Levenshtein
 * recurrence: D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1,
 * D[i-1][j-1] + [a_i != b_j]).
 */
#include <stdint.h>
#include <stdlib.h>

/* Full O(la*lb) dynamic program, two rows. */
int32_t oracle_edit_distance(const uint8_t *a, int32_t la, const uint8_t *b, int32_t lb) {
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    for (int32_t j = 0; j <= lb; j++) prev[j] = j;
    for (int32_t i = 1; i <= la; i++) {
        cur[0] = i;
        for (int32_t j = 1; j <= lb; j++) {
            int32_t v = prev[j - 1] + (a[i - 1] != b[j - 1]);
            if (prev[j] + 1 < v) v = prev[j] + 1;
            if (cur[j - 1] + 1 < v) v = cur[j - 1] + 1;
            cur[j] = v;
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    int32_t r = prev[lb];
    free(prev); free(cur);
    return r;
}

/*
 * Banded form (Ukkonen): only cells with |i - j| <= k are computed, cells
 * outside the band count as k + 1.  Returns the distance if it is <= k,
 * else -1 (the threshold form the paper uses for labelling).
 */
int32_t oracle_edit_distance_banded(const uint8_t *a, int32_t la, const uint8_t *b, int32_t lb, int32_t k) {
    if (k < 0) return -1;
    int32_t diff = la > lb ? la - lb : lb - la;
    if (diff > k) return -1;
    const int32_t INF = k + 1;
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    for (int32_t j = 0; j <= lb; j++) prev[j] = j <= k ? j : INF;
    for (int32_t i = 1; i <= la; i++) {
        int32_t lo = i - k > 1 ? i - k : 1, hi = i + k < lb ? i + k : lb;
        for (int32_t j = 0; j <= lb; j++) cur[j] = INF;
        cur[0] = i <= k ? i : INF;
        for (int32_t j = lo; j <= hi; j++) {
            int32_t v = prev[j - 1] + (a[i - 1] != b[j - 1]);
            if (prev[j] + 1 < v) v = prev[j] + 1;
            if (cur[j - 1] + 1 < v) v = cur[j - 1] + 1;
            cur[j] = v < INF ? v : INF;
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    int32_t r = prev[lb];
    free(prev); free(cur);
    return r <= k ? r : -1;
}

/* Threshold labels for n equal-length pairs (rows at p * stride). */
int oracle_edit_distance_batch(const uint8_t *P, const uint8_t *T, int64_t stride,
                               const int32_t *lengths, int64_t n, const int32_t *k_per_pair,
                               int32_t k, int32_t *out) {
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < n; p++) {
        int32_t m = lengths[p], kk = k_per_pair ? k_per_pair[p] : k;
        out[p] = oracle_edit_distance_banded(P + p * stride, m, T + p * stride, m, kk);
    }
    return 0;
}
