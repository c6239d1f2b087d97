/*
 * CPU ORACLE for the Shouji pre-alignment filter -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, character-level implementation used to check the GPU path.
 * Only tests, the smoke check and the bench's CPU-baseline leg may load it;
 * the product path never calls it.  It shares no code with the GPU library:
 * it reads base codes (one uint8 per base), never the packed device layout.
 *
 * Source: Alser et al., "Shouji: a fast and efficient pre-alignment filter
 * for sequence alignment", Sec. 2.2 (three steps), Eq. 1 (neighbourhood map),
 * Supplementary Sec. 6.2 Algorithm 1 and Algorithm 2 (CZ, count zeros).
 *
 * Readings adopted where the paper is ambiguous (each is listed with its
 * evidence in the design notes):
 *  - Pattern P = read, text T = reference; map entry N[i][j] compares P[i]
 *    with T[j] (Eq. 1).  A diagonal d is viewed along the text column j:
 *    cell (d, j) compares P[j-d] with T[j]; d > 0 are the upper diagonals
 *    (pattern shifted right, Sec. 2.3), d < 0 the lower ones, d = 0 main.
 *  - Cells outside the m x m map (j-d or j outside [0, m)) count as
 *    mismatches (1), which also makes the last three windows of the m
 *    windows (Sec. 2.2.2: one window per column, width 4, step 1) see ones
 *    beyond column m-1.
 *  - Window search: every one of the 2E+1 diagonal segments is examined
 *    (Sec. 2.2.2); the winner has the most zeros, ties going to a segment
 *    that starts with a zero; remaining ties go to the earliest segment in
 *    Algorithm 1's evaluation order ("reading B"): for j = 1..E the j-th
 *    diagonal whose text index exceeds the pattern index by j (Algorithm 1
 *    indexes the map by text row and pattern column and calls it the lower
 *    one; it is d = +j here and "Upper Diagonal-j" in Fig. 6), then the one
 *    with d = -j, and the main diagonal last.  Fig. 6(c)'s local count of 2
 *    needs this order (the opposite order gives 3).  Reading A (off-diagonals
 *    first, then the main diagonal replaces the winner only with strictly
 *    more zeros, as Algorithm 1's final comparison is written) is kept behind
 *    a flag for sensitivity studies only.
 *  - Shouji bit-vector update: copy the winner into S[i..i+3] only when it
 *    has strictly more zeros than S[i..i+3] (Algorithm 1's update test).
 *  - Decision: accept (1) iff the number of ones in S[0..m) is <= E
 *    (Sec. 2.2.3; Algorithm 1's test CZ(S) >= m - E).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Neighbourhood map entry (Eq. 1) on diagonal d at text column j, for a
 * pattern of length mP and a text of length mT. */
static int map_cell2(const uint8_t *P, int mP, const uint8_t *T, int mT, int d, int j) {
    int q = j - d;                         /* pattern index on this diagonal */
    if (j < 0 || j >= mT || q < 0 || q >= mP) return 1;
    return P[q] == T[j] ? 0 : 1;
}

static int map_cell(const uint8_t *P, const uint8_t *T, int m, int d, int j) {
    return map_cell2(P, m, T, m, d, j);
}

/* One diagonal row of the map (Eq. 1): out[j] = cell (d, j) for j in [0, m). */
int oracle_shouji_map_row(const uint8_t *P, const uint8_t *T, int32_t m, int32_t d, uint8_t *out) {
    if (m < 0) return -1;
    for (int j = 0; j < m; j++) out[j] = (uint8_t)map_cell(P, T, m, d, j);
    return 0;
}

/* CZ (Algorithm 2): zeros in a bit-vector of length len. */
static int count_zeros(const uint8_t *v, int len) {
    int c = 0;
    for (int t = 0; t < len; t++) if (v[t] == 0) c++;
    return c;
}

/*
 * Steps 1 and 2 of the filter (Sec. 2.2.1-2.2.2; Algorithm 1) for a pattern
 * P of length mP and a text T of length mT with windows of W columns (W = 4
 * in Shouji; other widths only for the window-width study of Suppl. Sec.
 * 6.1).  Every other form of the filter in this file calls this one
 * function, so the worked examples that pin any of them pin all of them.
 * On return S[0 .. mT+W-2] holds the Shouji bit-vector (positions >= mT
 * stay 1).  reading: 0 = B (the adopted reading), 1 = A (sensitivity study
 * only).
 */
static void shouji_steps(const uint8_t *P, int mP, const uint8_t *T, int mT, int E, int W, int reading,
                         uint8_t *S) {
    /* Step 1 (Sec. 2.2.1): the 2E+1 diagonals, stored as rows over text
     * columns 0 .. mT+W-2 so that every window i in [0, mT) reads W cells. */
    int nd = 2 * E + 1, w = mT + W - 1;
    uint8_t *N = (uint8_t *)malloc((size_t)nd * (size_t)w + 1);
    for (int d = -E; d <= E; d++)
        for (int j = 0; j < w; j++)
            N[(size_t)(d + E) * w + j] = (uint8_t)map_cell2(P, mP, T, mT, d, j);
    /* Step 2 (Sec. 2.2.2): the Shouji bit-vector starts as all ones; one
     * window per text column. */
    for (int j = 0; j < w; j++) S[j] = 1;
    for (int i = 0; i < mT; i++) {
        const uint8_t *Z = NULL;
        int best_key = -1;
        /* off-diagonal candidates in evaluation order d = +1, -1, ..., +E, -E;
         * key = 2 * zeros + leading zero, the earliest keeps full ties */
        for (int k = 1; k <= E; k++) {
            for (int s = 0; s < 2; s++) {
                int d = s == 0 ? k : -k;
                const uint8_t *seg = N + (size_t)(d + E) * w + i;
                int key = 2 * count_zeros(seg, W) + (seg[0] == 0 ? 1 : 0);
                if (key > best_key) { best_key = key; Z = seg; }
            }
        }
        const uint8_t *M = N + (size_t)E * w + i;     /* main diagonal, last */
        if (reading == 0) {
            int key = 2 * count_zeros(M, W) + (M[0] == 0 ? 1 : 0);
            if (key > best_key) { best_key = key; Z = M; }
        } else {
            if (Z == NULL || count_zeros(M, W) > count_zeros(Z, W)) Z = M;
        }
        /* update S[i..i+W-1] only with strictly more zeros */
        if (count_zeros(Z, W) > count_zeros(S + i, W))
            for (int t = 0; t < W; t++) S[i + t] = Z[t];
    }
    free(N);
}

/*
 * Filter one pair.  P, T: base codes, length m (>= 0).  reading: 0 = B (the
 * adopted reading), 1 = A (sensitivity study only).  If S_out is not NULL it
 * receives the final Shouji bit-vector S[0..m).  Returns the number of ones.
 */
int oracle_shouji_pair(const uint8_t *P, const uint8_t *T, int32_t m, int32_t E,
                       int32_t reading, uint8_t *S_out) {
    if (m < 0 || E < 0) return -1;
    uint8_t *S = (uint8_t *)malloc((size_t)m + 4);
    shouji_steps(P, m, T, m, E, 4, reading, S);
    /* Step 3 (Sec. 2.2.3): count the ones over the m positions. */
    int ones = 0;
    for (int j = 0; j < m; j++) ones += S[j];
    if (S_out) memcpy(S_out, S, (size_t)m);
    free(S);
    return ones;
}

/*
 * Window width W instead of 4 (Suppl. Sec. 6.1, Fig. 4 compares widths): the
 * same steps with W-column windows: every window i in [0, m) examines the
 * W-bit segment of each diagonal at text columns i..i+W-1, the winner (most
 * zeros, then a leading zero, then the evaluation order) is copied into
 * S[i..i+W-1] when it has strictly more zeros, and the ones of S[0..m) are
 * counted.  W = 4 is oracle_shouji_pair.  Returns the ones (or -1).
 */
int oracle_shouji_pair_w(const uint8_t *P, const uint8_t *T, int32_t m, int32_t E, int32_t W,
                         uint8_t *S_out) {
    if (m < 0 || E < 0 || W < 1) return -1;
    uint8_t *S = (uint8_t *)malloc((size_t)m + (size_t)W);
    shouji_steps(P, m, T, m, E, W, 0, S);
    int ones = 0;
    for (int j = 0; j < m; j++) ones += S[j];
    if (S_out) memcpy(S_out, S, (size_t)m);
    free(S);
    return ones;
}

int oracle_shouji_batch_w(const uint8_t *P, const uint8_t *T, int64_t stride, const int32_t *lengths,
                          int64_t n, int32_t E, int32_t W, int32_t nthreads, uint8_t *out_accept,
                          int16_t *out_popcount) {
    if (n < 0 || stride < 0 || E < 0 || W < 1) return -1;
    #pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int64_t p = 0; p < n; p++) {
        int32_t m = lengths[p];
        if (m < 0 || m > stride) {
            out_accept[p] = 0xFF;
            if (out_popcount) out_popcount[p] = -1;
            continue;
        }
        int ones = oracle_shouji_pair_w(P + p * stride, T + p * stride, m, E, W, NULL);
        out_accept[p] = (uint8_t)(ones <= E ? 1 : 0);
        if (out_popcount) out_popcount[p] = (int16_t)ones;
    }
    return 0;
}

/*
 * Counting modes of the final step (Sec. 2.2.3: local filtering ignores the
 * ones at both ends of the bit-vector, glocal filtering those at one end;
 * Suppl. Sec. 8, Fig. 6(c)).  The ones "at an end" are the run of ones
 * before the first zero (start) or after the last zero (end).  A vector
 * without any zero keeps all its ones in every mode.
 */
enum { ORACLE_GLOBAL = 0, ORACLE_LOCAL = 1, ORACLE_GLOCAL_START = 2, ORACLE_GLOCAL_END = 3 };

/*
 * Filter one pair of possibly different lengths: pattern (read) P of length
 * mP, text (reference) T of length mT.  The map has the text's mT columns,
 * so there are mT windows and the bit-vector spans text positions [0, mT);
 * cells whose pattern index leaves [0, mP) are mismatches, as above.  The
 * steps are those of oracle_shouji_pair; only the final count depends on
 * `mode`.  S_out (may be NULL) receives S[0..mT).  Returns the count.
 */
int oracle_shouji_pair2(const uint8_t *P, int32_t mP, const uint8_t *T, int32_t mT, int32_t E,
                        int32_t mode, int32_t reading, uint8_t *S_out) {
    if (mP < 0 || mT < 0 || E < 0 || mode < 0 || mode > 3) return -1;
    uint8_t *S = (uint8_t *)malloc((size_t)mT + 4);
    shouji_steps(P, mP, T, mT, E, 4, reading, S);
    /* Step 3 with the counting mode: the range of positions whose ones count */
    int first = -1, last = -1;
    for (int j = 0; j < mT; j++)
        if (S[j] == 0) { if (first < 0) first = j; last = j; }
    int lo = 0, hi = mT;                    /* count over [lo, hi) */
    if (first >= 0) {
        if (mode == ORACLE_LOCAL || mode == ORACLE_GLOCAL_START) lo = first;
        if (mode == ORACLE_LOCAL || mode == ORACLE_GLOCAL_END) hi = last + 1;
    }
    int ones = 0;
    for (int j = lo; j < hi; j++) ones += S[j];
    if (S_out) memcpy(S_out, S, (size_t)mT);
    free(S);
    return ones;
}

/*
 * Batch form of oracle_shouji_pair2: row p of P and T starts at p * stride;
 * read_lengths[p] = mP, ref_lengths[p] = mT; a length outside [0, stride] or
 * a negative threshold marks the pair invalid (0xFF / -1).
 */
int oracle_shouji_batch2(const uint8_t *P, const uint8_t *T, int64_t stride,
                         const int32_t *read_lengths, const int32_t *ref_lengths, int64_t n,
                         int32_t E, const int32_t *E_per_pair, int32_t mode, int32_t nthreads,
                         uint8_t *out_accept, int16_t *out_popcount) {
    if (n < 0 || stride < 0 || (E < 0 && !E_per_pair) || mode < 0 || mode > 3) return -1;
    #pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int64_t p = 0; p < n; p++) {
        int32_t mP = read_lengths[p], mT = ref_lengths[p], e = E_per_pair ? E_per_pair[p] : E;
        if (mP < 0 || mP > stride || mT < 0 || mT > stride || e < 0) {
            out_accept[p] = 0xFF;
            if (out_popcount) out_popcount[p] = -1;
            continue;
        }
        int ones = oracle_shouji_pair2(P + p * stride, mP, T + p * stride, mT, e, mode, 0, NULL);
        out_accept[p] = (uint8_t)(ones <= e ? 1 : 0);
        if (out_popcount) out_popcount[p] = (int16_t)ones;
    }
    return 0;
}

/*
 * Filter n pairs.  Row p of P and T starts at p * stride (codes).  lengths[p]
 * is the pair's length; a length outside [0, stride] marks an invalid pair:
 * out_accept = 0xFF, out_popcount = -1.  Threshold E, or E_per_pair[p] when
 * E_per_pair is not NULL (a negative entry also marks the pair invalid).
 * out_popcount may be NULL.  nthreads <= 0 uses the OpenMP default.
 */
int oracle_shouji_batch(const uint8_t *P, const uint8_t *T, int64_t stride,
                        const int32_t *lengths, int64_t n, int32_t E,
                        const int32_t *E_per_pair, int32_t reading, int32_t nthreads,
                        uint8_t *out_accept, int16_t *out_popcount) {
    if (n < 0 || stride < 0 || (E < 0 && !E_per_pair)) return -1;
    if (nthreads > 0) {
        #pragma omp parallel for schedule(static) num_threads(nthreads)
        for (int64_t p = 0; p < n; p++) {
            int32_t m = lengths[p], e = E_per_pair ? E_per_pair[p] : E;
            if (m < 0 || m > stride || e < 0) { out_accept[p] = 0xFF; if (out_popcount) out_popcount[p] = -1; continue; }
            int ones = oracle_shouji_pair(P + p * stride, T + p * stride, m, e, reading, NULL);
            out_accept[p] = (uint8_t)(ones <= e ? 1 : 0);
            if (out_popcount) out_popcount[p] = (int16_t)ones;
        }
    } else {
        #pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; p++) {
            int32_t m = lengths[p], e = E_per_pair ? E_per_pair[p] : E;
            if (m < 0 || m > stride || e < 0) { out_accept[p] = 0xFF; if (out_popcount) out_popcount[p] = -1; continue; }
            int ones = oracle_shouji_pair(P + p * stride, T + p * stride, m, e, reading, NULL);
            out_accept[p] = (uint8_t)(ones <= e ? 1 : 0);
            if (out_popcount) out_popcount[p] = (int16_t)ones;
        }
    }
    return 0;
}

/* Number of threads an OpenMP parallel region uses by default here. */
int oracle_default_threads(void) {
    int t = 1;
    #pragma omp parallel
    {
        #pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}
