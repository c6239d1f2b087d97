/*
 * Seeded synthetic read / reference-segment pairs for the Shouji filter.
 *
 * Shared by the CPU oracle's tests and by the GPU path's tests and bench: this
 * file holds no step of the filter itself, only random sequences and edits.
 * Inputs stand in for the paper's mrFAST-generated candidate pairs (Sec. 3.1,
 * Tables 5-8), which are not available: reads of length m, references made
 * from the read by k random edits, and a share of unrelated pairs.
 *
 * Random numbers: xoshiro256** seeded through splitmix64 (Blackman & Vigna,
 * public-domain published algorithms).  Each pair draws from its own stream,
 * seeded from (seed, pair index), so generation is parallel and reproducible.
 *
 * Base codes: 0..3 (A, C, G, T); only equality of codes matters downstream.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t next_u64(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl64(s[3], 45);
    return result;
}
static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ (0xD1B54A32D192ED03ULL * (stream + 1));
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
/* uniform integer in [0, n) (multiply-shift; bias below 2^-32 for our n) */
static uint32_t uni(rng_t *r, uint32_t n) {
    return (uint32_t)(((unsigned __int128)next_u64(r) * n) >> 64);
}
static double u01(rng_t *r) { return (double)(next_u64(r) >> 11) * (1.0 / 9007199254740992.0); }

/*
 * Generate n pairs into row-major code buffers (row p at p * stride).
 *   m_min..m_max  : read length drawn uniformly (equal bounds: fixed length)
 *   E_fixed >= 0  : threshold used to draw the edit count; else per pair
 *                   E_p = floor(r * m) with r uniform in [0, r_max]
 *   p_unrelated   : probability that the reference is an independent random sequence
 *   p_repeat      : probability of one tandem-repeat block in the read
 *                   (period 1..6, covering 20-60% of the read)
 * The reference is the read with k ~ U{0..2E_p} edits applied one after another
 * (substitution / insertion / deletion with probability 1/3 each, uniform
 * position), then truncated or padded with random bases to the read's length.
 * Outputs: P (reads), T (references), lengths, E_out (per pair threshold).
 */
int syn_generate(uint64_t seed, int64_t n, int32_t m_min, int32_t m_max, int64_t stride,
                 int32_t E_fixed, double r_max, double p_unrelated, double p_repeat,
                 uint8_t *P, uint8_t *T, int32_t *lengths, int32_t *E_out) {
    if (n < 0 || m_min < 0 || m_max < m_min || stride < m_max) return -1;
    #pragma omp parallel
    {
        uint8_t *buf = (uint8_t *)malloc((size_t)(3 * m_max + 16));
        #pragma omp for schedule(static)
        for (int64_t p = 0; p < n; p++) {
            rng_t r; rng_seed(&r, seed, (uint64_t)p);
            uint8_t *rd = P + p * stride, *rf = T + p * stride;
            memset(rd, 0, (size_t)stride); memset(rf, 0, (size_t)stride);
            int32_t m = m_min + (int32_t)uni(&r, (uint32_t)(m_max - m_min + 1));
            int32_t E = E_fixed >= 0 ? E_fixed : (int32_t)floor(u01(&r) * r_max * m);
            lengths[p] = m; if (E_out) E_out[p] = E;
            for (int32_t j = 0; j < m; j++) rd[j] = (uint8_t)uni(&r, 4);
            if (u01(&r) < p_repeat && m > 0) {
                int32_t q = 1 + (int32_t)uni(&r, 6);
                uint8_t unit[6];
                for (int t = 0; t < q; t++) unit[t] = (uint8_t)uni(&r, 4);
                double f = 0.2 + 0.4 * u01(&r);
                int32_t L = (int32_t)floor(f * m);
                int32_t start = (int32_t)uni(&r, (uint32_t)(m - L + 1));
                for (int32_t t = 0; t < L; t++) rd[start + t] = unit[t % q];
            }
            if (u01(&r) < p_unrelated) {
                for (int32_t j = 0; j < m; j++) rf[j] = (uint8_t)uni(&r, 4);
                continue;
            }
            int32_t k = (int32_t)uni(&r, (uint32_t)(2 * E + 1));
            int32_t len = m;
            memcpy(buf, rd, (size_t)m);
            for (int32_t e = 0; e < k; e++) {
                uint32_t op = uni(&r, 3);
                if (op == 0) {                      /* substitution by another base */
                    if (len == 0) continue;
                    int32_t pos = (int32_t)uni(&r, (uint32_t)len);
                    buf[pos] = (uint8_t)((buf[pos] + 1 + uni(&r, 3)) & 3);
                } else if (op == 1) {               /* insertion */
                    if (len >= 3 * m_max + 15) continue;
                    int32_t pos = (int32_t)uni(&r, (uint32_t)(len + 1));
                    memmove(buf + pos + 1, buf + pos, (size_t)(len - pos));
                    buf[pos] = (uint8_t)uni(&r, 4);
                    len++;
                } else {                            /* deletion */
                    if (len == 0) continue;
                    int32_t pos = (int32_t)uni(&r, (uint32_t)len);
                    memmove(buf + pos, buf + pos + 1, (size_t)(len - pos - 1));
                    len--;
                }
            }
            for (int32_t j = 0; j < m; j++) rf[j] = j < len ? buf[j] : (uint8_t)uni(&r, 4);
        }
        free(buf);
    }
    return 0;
}

/*
 * Serving-pool variant: pairs whose reference segment is read out of one shared
 * pool of random bases at a per-pair offset, and whose read is an edited copy of
 * that segment (or unrelated).  pool holds pool_len codes (generated here from
 * the seed).  Offsets are written to off_out.
 */
int syn_pool(uint64_t seed, int64_t pool_len, uint8_t *pool) {
    if (pool_len < 0) return -1;
    const int64_t blk = 1 << 16;
    int64_t nb = (pool_len + blk - 1) / blk;
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; b++) {
        rng_t r; rng_seed(&r, seed ^ 0x5EEDF00DULL, (uint64_t)b);
        int64_t hi = (b + 1) * blk < pool_len ? (b + 1) * blk : pool_len;
        for (int64_t j = b * blk; j < hi; j++) pool[j] = (uint8_t)uni(&r, 4);
    }
    return 0;
}
