/*
 * CPU ORACLE for the MAGNET pre-alignment filter -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, character-level implementation used to check the GPU path;
 * only tests and the bench's oracle samples load it.  It shares no code with
 * the GPU library (base codes, one uint8 per base).
 *
 * Source: Shouji paper, Supplementary Sec. 7.1 (MAGNET overview, five steps),
 * Algorithm 3 (MAGNET) and Algorithm 4 (the EXEN function).  The steps are
 * taken in the paper's order: build the 2E+1 diagonal bit-vectors of the
 * neighbourhood map; start the MAGNET bit-vector as all ones; EXEN over the
 * whole sequence: extract the longest run of consecutive zeros among all
 * diagonals, stop at once in the first call if it is shorter than
 * ceil((m-E)/(E+1)), record it as zeros of the MAGNET vector, and recurse on
 * the right part (after the run and one more encapsulating position) and
 * then the left part (before the run and one encapsulating position), with
 * at most E+1 runs extracted in all; accept iff the MAGNET vector has at
 * least m-E zeros.
 *
 * Readings adopted where the text and the listings are silent or loose (each
 * is listed with its evidence in the design notes):
 *  - Diagonals share Shouji's map (Eq. 1): one vector per diagonal d in
 *    [-E, E] indexed by text position j, cell (d, j) = [P[j-d] != T[j]],
 *    cells outside the map are ones.  d = +k is the diagonal the listings
 *    call "lower" (text index = pattern index + k, the listings index the
 *    map by text row and pattern column), d = -k the "upper" one.  A
 *    subproblem [SI, EI] is a range of text positions searched on every
 *    diagonal; for the first call the listing's starting cells are exactly
 *    the first cells of each diagonal inside the map.
 *  - The extraction keeps one global longest run.  For k = 1..E the lower
 *    run replaces the upper one of the same k only when strictly longer
 *    (Algorithm 4's "X > Y" test), the pair's pick replaces the run kept so
 *    far only when strictly longer (so the smallest k wins ties), and the
 *    main diagonal replaces it only when strictly longer (the listing's
 *    final test).  Within one diagonal the leftmost of equally long runs.
 *  - A run found is written as zeros into the MAGNET vector (the listing
 *    leaves this store implicit; the overview says the run's length is kept
 *    toward the total).  A subproblem in which no diagonal has a zero
 *    extracts nothing and returns as an empty one does (calls - 1).
 *  - The first call's early exit leaves the vector all ones (the pair is
 *    rejected whenever m > E; with m <= E the threshold is not positive).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Neighbourhood map entry (Eq. 1) on diagonal d at text position j. */
static int cell(const uint8_t *P, const uint8_t *T, int m, int d, int j) {
    int q = j - d;
    if (j < 0 || j >= m || q < 0 || q >= m) return 1;
    return P[q] == T[j] ? 0 : 1;
}

typedef struct {
    const uint8_t *N;   /* 2E+1 rows (d + E) of m cells */
    int m, E;
    int a;              /* ceil((m-E)/(E+1)), 0 when m <= E */
    uint8_t *V;         /* MAGNET bit-vector */
} magnet_state;

/* CCZ: the longest run of zeros of diagonal d inside [lo, hi] (leftmost of
 * equal ones).  Returns its length (0 if none), start in *s. */
static int ccz(const magnet_state *st, int d, int lo, int hi, int *s) {
    const uint8_t *row = st->N + (size_t)(d + st->E) * (size_t)st->m;
    int best = 0, run = 0;
    *s = -1;
    for (int j = lo; j <= hi; j++) {
        if (row[j] == 0) {
            run++;
            if (run > best) { best = run; *s = j - run + 1; }
        } else {
            run = 0;
        }
    }
    return best;
}

/* EXEN (Algorithm 4) on text positions [SI, EI]; returns the updated count
 * of calls. */
static int exen(magnet_state *st, int SI, int EI, int calls) {
    if (SI <= EI && calls <= st->E + 1) {
        /* Step 2: extraction of the longest run over all diagonals */
        int len = 0, s = -1;
        for (int k = 1; k <= st->E; k++) {
            int s1, s2;
            int X = ccz(st, +k, SI, EI, &s1);    /* lower diagonal */
            int Y = ccz(st, -k, SI, EI, &s2);    /* upper diagonal */
            int pl = X > Y ? X : Y, ps = X > Y ? s1 : s2;
            if (pl > len) { len = pl; s = ps; }
        }
        int s0;
        int X = ccz(st, 0, SI, EI, &s0);         /* main diagonal */
        if (X > len) { len = X; s = s0; }
        /* early termination, first call only */
        if (calls == 1 && len < st->a) return 0;
        if (len == 0) return calls - 1;          /* no zero in this part */
        int e = s + len - 1;
        for (int j = s; j <= e; j++) st->V[j] = 0;
        /* Steps 3-4: encapsulate the run, right part first, then left */
        calls = exen(st, e + 2, EI, calls + 1);
        calls = exen(st, SI, s - 2, calls + 1);
        return calls;
    }
    return calls - 1;
}

/*
 * MAGNET on one equal-length pair.  P, T: base codes, length m >= 0.  If
 * V_out is not NULL it receives the final MAGNET bit-vector V[0..m).
 * Returns the number of ones of V (accept iff <= E), or -1.
 */
int oracle_magnet_pair(const uint8_t *P, const uint8_t *T, int32_t m, int32_t E, uint8_t *V_out) {
    if (m < 0 || E < 0) return -1;
    magnet_state st;
    st.m = m;
    st.E = E;
    st.a = m > E ? (m - E + (E + 1) - 1) / (E + 1) : 0;   /* ceil((m-E)/(E+1)) */
    uint8_t *N = (uint8_t *)malloc((size_t)(2 * E + 1) * (size_t)m + 1);
    st.V = (uint8_t *)malloc((size_t)m + 1);
    /* Step 1: the 2E+1 diagonal bit-vectors */
    for (int d = -E; d <= E; d++)
        for (int j = 0; j < m; j++) N[(size_t)(d + E) * (size_t)m + j] = (uint8_t)cell(P, T, m, d, j);
    st.N = N;
    for (int j = 0; j < m; j++) st.V[j] = 1;
    exen(&st, 0, m - 1, 1);
    /* Step 5: count */
    int ones = 0;
    for (int j = 0; j < m; j++) ones += st.V[j];
    if (V_out) memcpy(V_out, st.V, (size_t)m);
    free(N);
    free(st.V);
    return ones;
}

int oracle_magnet_batch(const uint8_t *P, const uint8_t *T, int64_t stride, const int32_t *lengths, int64_t n,
                        int32_t E, int32_t nthreads, uint8_t *out_accept, int16_t *out_popcount) {
    if (n < 0 || stride < 0 || E < 0) return -1;
    #pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int64_t p = 0; p < n; p++) {
        int32_t m = lengths[p];
        if (m < 0 || m > stride) {
            out_accept[p] = 0xFF;
            if (out_popcount) out_popcount[p] = -1;
            continue;
        }
        int ones = oracle_magnet_pair(P + p * stride, T + p * stride, m, E, NULL);
        out_accept[p] = (uint8_t)(ones <= E ? 1 : 0);
        if (out_popcount) out_popcount[p] = (int16_t)ones;
    }
    return 0;
}
