/*
 * shouji.h -- C ABI of the MI355X Shouji pre-alignment filter.
 *
 * The filter (Alser et al., Shouji, Sec. 2.2; Supplementary Algorithm 1)
 * decides for each read / reference-segment pair whether it may lie within
 * E edits: it builds the 2E+1 diagonals of the neighbourhood map (Eq. 1),
 * slides a 4-column window over them, copies into the Shouji bit-vector the
 * diagonal segment with the most matches, and accepts the pair when that
 * vector keeps at most E ones (Sec. 2.2.3).  Accepted pairs go on to full
 * alignment; rejected pairs need none.
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer on the current HIP device.  The
 *    caller owns all buffers; the library keeps no pointer after returning.
 *  - Sequences are 2-bit packed, 16 bases per 32-bit word, base j of a
 *    sequence in bits [2*(j%16), 2*(j%16)+1] of word j/16.  Any fixed code
 *    assignment works (only equality of codes is tested); the reference
 *    generator uses A=0, C=1, G=2, T=3.  Words are stored word-major:
 *    word w of pair p is at seq[w * ld + p], ld >= n_pairs (so one load
 *    instruction of a wavefront reads one word of 64 consecutive pairs).
 *    Words needed per pair: ceil(max_len / 16).  Bits beyond a pair's
 *    length are ignored.
 *  - The read is the pattern P and the reference segment the text T of
 *    Eq. 1; read and reference of a pair have the same length (global
 *    filtering, Sec. 2.3).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and results are valid after the stream is synchronised.  Argument
 *    errors are detected on the host before anything is enqueued.
 *  - Functions return SHOUJI_OK or a negative shouji_status and never throw.
 *    shouji_last_error() returns a thread-local description of the last
 *    failure.
 *  - Per-pair problems (a length outside [0, max_len]) do not fail the call:
 *    that pair gets out_accept = 0xFF and out_popcount = -1.
 *  - Thread-safe and re-entrant; calls on different streams may overlap.
 */
#ifndef SHOUJI_H
#define SHOUJI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHOUJI_BASES_PER_WORD 16
#define SHOUJI_MAX_LEN 1024 /* longest supported sequence (bases)            */
#define SHOUJI_MAX_E 31     /* largest edit threshold after clamping to m-1  */
#define SHOUJI_MAX_WINDOW 16 /* widest window of shouji_filter_window        */

typedef enum {
    SHOUJI_OK = 0,
    SHOUJI_ERR_NULL = -1,   /* a required pointer is NULL                    */
    SHOUJI_ERR_ARG = -2,    /* a size or stride is invalid                   */
    SHOUJI_ERR_RANGE = -3,  /* E or max_len beyond the supported maximum     */
    SHOUJI_ERR_DEVICE = -4, /* the HIP runtime reported an error             */
    SHOUJI_ERR_NOMEM = -5   /* a device allocation failed                    */
} shouji_status;

/*
 * shouji_filter -- the plain form: one edit threshold for every pair.
 *
 * Sec. 2.2 (Steps 1-3), Eq. 1, Supplementary Algorithm 1.  Per pair p:
 *   Step 1: diagonal d in [-E, E] at text column j is 0 iff
 *           0 <= j, j-d < m and read[j-d] == ref[j], else 1;
 *   Step 2: S = all ones; for each window i in [0, m) the segment of
 *           columns i..i+3 with the most zeros wins (ties: a leading zero,
 *           then the order d = +1, -1, +2, -2, ..., +E, -E, 0: Algorithm 1
 *           examines first the diagonal whose text index exceeds the
 *           pattern index by j, i.e. d = +j);
 *           it is copied into S[i..i+3] if it has strictly more zeros;
 *   Step 3: popcount = ones of S over [0, m); accept = popcount <= E.
 *
 *   reads, refs   word-major packed sequences (see above), ld words apart.
 *   lengths       n_pairs lengths m_p, or NULL: every pair has max_len bases
 *                 (the faster call for equal lengths: its kernel keeps only the
 *                 pattern ring in LDS, two wavefronts per SIMD up to E = 22).
 *   E             edit threshold, >= 0.  Internally clamped to max_len - 1
 *                 (diagonals beyond the map are all ones); after clamping it
 *                 must be <= SHOUJI_MAX_E, else SHOUJI_ERR_RANGE.
 *   out_accept    n_pairs bytes: 1 accept, 0 reject, 0xFF invalid pair.
 *   out_popcount  n_pairs int16 ones counts (-1 for an invalid pair), or NULL.
 *   n_pairs       >= 0; 0 is a successful no-op.
 *   max_len       0..SHOUJI_MAX_LEN, the longest length in the batch.
 *   ld            leading dimension in words, >= n_pairs.
 *   stream        hipStream_t or NULL.
 * Nothing is allocated.  Above E = 13 with lengths (E = 22 without) the
 * kernel's wavefronts also post their progress in a 64 KB library-owned
 * device table per GPU, read only to set issue priority: calls that overlap
 * share it without any effect on their results.
 */
int shouji_filter(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                  int32_t E, uint8_t *out_accept, int16_t *out_popcount,
                  int64_t n_pairs, int32_t max_len, int64_t ld, void *stream);

/*
 * Relayout into the filters' input layout.
 *
 * The bases are stored in 2 bits each (Sec. 2.3: the filter streams four
 * bases per byte of its link).  This converts sequences kept pair by pair,
 * 32 bases per 64-bit word, into the word-major 16-base layout above (row r
 * of a sequence, bases 16r..16r+15, at r * ld + p), on the device.
 *
 *   src           n_pairs * words_per_seq uint64 (device): pair p's words at
 *                 src[p * words_per_seq + w], base j of the sequence in bits
 *                 2(j mod 32)..2(j mod 32)+1 of its word j / 32 (the code of
 *                 each base is kept as it is: only equality matters).
 *   words_per_seq >= ceil(max_len / 32), else SHOUJI_ERR_ARG.
 *   n_pairs       >= 0; 0 is a successful no-op.
 *   max_len       0..SHOUJI_MAX_LEN: dst receives ceil(max_len / 16) rows.
 *   dst           ceil(max_len / 16) rows of ld uint32 (device), written for
 *                 pairs 0..n_pairs-1 (other columns untouched); owned by the
 *                 caller, nothing is allocated.
 *   ld            leading dimension of dst in words, >= n_pairs.
 *   stream        hipStream_t or NULL.
 * Call it once for the reads and once for the references.  Errors
 * (SHOUJI_ERR_ARG / _RANGE / _NULL) are reported before anything is launched.
 */
int shouji_relayout_pair_major(const uint64_t *src, int64_t words_per_seq, int64_t n_pairs, int32_t max_len,
                               uint32_t *dst, int64_t ld, void *stream);

/*
 * Two-length form: reads and reference segments of different lengths, and
 * local or glocal counting.
 *
 * Sec. 2.2.3 (local filtering leaves out the ones at both ends of the Shouji
 * bit-vector, glocal filtering those at one end), Suppl. Sec. 8 and Fig. 6(c)
 * (a read shorter than its reference segment).  Per pair p with read length
 * mP = read_lengths[p] and reference length mT = ref_lengths[p]:
 *   Step 1: cell (d, j) for text (reference) column j in [0, mT) is 0 iff
 *           0 <= j-d < mP and read[j-d] == ref[j], else 1;
 *   Step 2: as for shouji_filter, over the mT windows of the reference;
 *   Step 3: count the ones of S over [0, mT), leaving out, when S has a
 *           zero, the ones before its first zero (modes LOCAL and
 *           GLOCAL_START) and after its last zero (LOCAL and GLOCAL_END);
 *           a vector without zeros keeps all its ones.  accept = count <= E.
 * With mP == mT and mode GLOBAL the results equal shouji_filter's.
 *
 *   read_lengths, ref_lengths  n_pairs lengths each (device, required); a
 *                 pair with either length outside [0, max_len] gets the
 *                 sentinels 0xFF / -1.
 *   mode          one of shouji_count_mode; else SHOUJI_ERR_ARG.
 *   max_len       the longest of all read and reference lengths; both
 *                 sequences of a pair hold ceil(max_len/16) words.
 *   other arguments and errors as for shouji_filter (out_popcount receives
 *                 the count of the chosen mode).
 */
typedef enum {
    SHOUJI_COUNT_GLOBAL = 0,       /* every one of S[0..mT)                     */
    SHOUJI_COUNT_LOCAL = 1,        /* without the ones at both ends             */
    SHOUJI_COUNT_GLOCAL_START = 2, /* without the ones before the first zero    */
    SHOUJI_COUNT_GLOCAL_END = 3    /* without the ones after the last zero      */
} shouji_count_mode;

int shouji_filter_local(const uint32_t *reads, const uint32_t *refs, const int32_t *read_lengths,
                        const int32_t *ref_lengths, int32_t E, int32_t mode, uint8_t *out_accept,
                        int16_t *out_popcount, int64_t n_pairs, int32_t max_len, int64_t ld,
                        void *stream);

/*
 * Batched form: mixed lengths and one edit threshold per pair in one pass.
 *
 * Same filter as shouji_filter (Sec. 2.2, Eq. 1, Algorithm 1) applied to every
 * pair with its own threshold E_per_pair[p]: results are identical to filtering
 * each pair alone.  Internally the pairs are grouped into bins of equal E and
 * similar length (a copy into the caller's workspace), the bins are cut into
 * tiles of up to 1024 pairs, and one kernel per E class filters all tiles,
 * writing results at the pairs' original indices.  Nothing is allocated and
 * every step is a kernel on `stream`, so a call can be captured in a graph
 * (the workspace contents are overwritten by every call).
 *
 *   reads, refs, lengths, ld, max_len, out_accept, out_popcount, n_pairs:
 *                 as for shouji_filter (lengths may be NULL).
 *   E_per_pair    n_pairs int32 thresholds (device).  A pair whose length is
 *                 outside [0, max_len], whose E is negative, or whose E after
 *                 clamping to m-1 exceeds SHOUJI_MAX_E gets the sentinels.
 *   workspace     device buffer of at least shouji_batched_workspace_bytes()
 *                 bytes, owned by the caller; one call at a time per buffer.
 *   config        tuning knobs, or NULL: the autotuned choice for this size
 *                 (shouji_tune_batched), else the defaults.
 */
typedef struct {
    int32_t bin_width;       /* length bucket in bases: 4, 8, 16 or 32 (0: default 8)  */
    int32_t waves_per_group; /* wavefronts per workgroup: 1, 2 or 4 (0: default 4)      */
} shouji_batched_config;

/* Workspace bytes shouji_filter_batched needs for n_pairs pairs of at most
 * max_len bases (any config); negative status on bad arguments.  The binning
 * indexes pairs in 32 bits: n_pairs above SHOUJI_MAX_BATCHED_PAIRS is
 * SHOUJI_ERR_RANGE here and in shouji_filter_batched. */
#define SHOUJI_MAX_BATCHED_PAIRS 2147483647LL
int64_t shouji_batched_workspace_bytes(int64_t n_pairs, int32_t max_len);

int shouji_filter_batched(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                          const int32_t *E_per_pair, uint8_t *out_accept, int16_t *out_popcount,
                          int64_t n_pairs, int32_t max_len, int64_t ld, void *workspace,
                          int64_t workspace_bytes, const shouji_batched_config *config,
                          void *stream);

/*
 * Autotuner of the batched form: runs every config (bin width x wavefronts
 * per workgroup) three times on these inputs, timed with events on `stream`
 * (the call synchronises the stream), keeps the fastest for this size class
 * (max_len / 64, log2 n_pairs) for later calls with config == NULL, and
 * returns it in *best (and its time in *best_ms).  Outputs hold the last run.
 */
int shouji_tune_batched(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                        const int32_t *E_per_pair, uint8_t *out_accept, int16_t *out_popcount,
                        int64_t n_pairs, int32_t max_len, int64_t ld, void *workspace,
                        int64_t workspace_bytes, void *stream, shouji_batched_config *best,
                        float *best_ms);

/*
 * Batched form that allocates nothing and takes no workspace.
 *
 * For callers that cannot allocate device memory: code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Filter, arguments,
 * results, sentinels and errors as for shouji_filter_batched; the binned copy
 * of the pairs lives in a device array owned by the library, of
 * SHOUJI_NOALLOC_SCRATCH_BYTES bytes, one per GPU the library runs on, held
 * until the process ends.  The call allocates nothing (no hipMalloc, no
 * allocating library routine).
 *
 *   n_pairs, max_len  the binned copy must fit the array:
 *                 shouji_batched_workspace_bytes(n_pairs, max_len) <=
 *                 SHOUJI_NOALLOC_SCRATCH_BYTES (about 780,000 pairs at
 *                 max_len 300, 1.8 million at max_len 100), else
 *                 SHOUJI_ERR_RANGE before anything is enqueued.
 *   Concurrency   every call on one GPU shares that GPU's array, which keeps
 *                 the last call's contents: calls that overlap on one GPU
 *                 (other streams, other threads) race and must be ordered by
 *                 the caller.  Counters the binning needs are cleared by its
 *                 own kernels in every call.
 */
#define SHOUJI_NOALLOC_SCRATCH_BYTES (128LL << 20)

int shouji_filter_batched_noalloc(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths,
                                  const int32_t *E_per_pair, uint8_t *out_accept, int16_t *out_popcount,
                                  int64_t n_pairs, int32_t max_len, int64_t ld,
                                  const shouji_batched_config *config, void *stream);

/*
 * Window-width variant: W-column search windows instead of 4.
 *
 * Suppl. Sec. 6.1 and Fig. 4 compare the accuracy of window widths (4 is the
 * paper's choice).  Same steps as shouji_filter with W in place of 4: window
 * i examines the W-bit segment of every diagonal at text columns i..i+W-1,
 * the winner (most zeros, then a leading zero, then the order of
 * shouji_filter) is copied into S[i..i+W-1] when it has strictly more zeros,
 * and accept = ones(S[0..m)) <= E.  With W = 4 the results equal
 * shouji_filter's.  Bit-sliced (32 pairs per register, 2048 pairs per
 * wavefront, every lane its own pairs); the LDS per wavefront grows with W
 * and E (pattern and text rings), so it runs fewer wavefronts per CU than
 * shouji_filter.
 *
 *   W             1..SHOUJI_MAX_WINDOW, else SHOUJI_ERR_RANGE.
 *   other arguments, sentinels and errors as for shouji_filter.
 */
int shouji_filter_window(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths, int32_t E,
                         int32_t W, uint8_t *out_accept, int16_t *out_popcount, int64_t n_pairs,
                         int32_t max_len, int64_t ld, void *stream);

/*
 * MAGNET: the divide-and-conquer filter of Suppl. Sec. 7.1 (Algorithms 3
 * and 4) over the same neighbourhood map (Eq. 1, diagonals indexed by text
 * position, cells outside the map are ones).
 *
 * Per pair: the longest run of zeros over all diagonals inside the whole
 * sequence is taken (per diagonal the leftmost of equal runs; across
 * diagonals the order d = -1, +1, ..., -E, +E, main, a later run replacing
 * the kept one only when strictly longer); if it is shorter than
 * ceil((m-E)/(E+1)) the pair is rejected with all m positions counted as
 * ones.  Otherwise it counts as matched, and the parts right of it and left
 * of it, each without the one position next to the run, are solved the same
 * way (right part first, no threshold), until E+1 runs are taken; a part with
 * no zero on any diagonal takes none.  popcount = m - total length of the
 * runs taken; accept = popcount <= E.  MAGNET rejects some pairs within E
 * (a single insertion costs 2), as the paper reports for it.
 *
 *   arguments, layout, sentinels and errors as for shouji_filter (E is
 *   clamped to m-1 for the diagonals only; E > SHOUJI_MAX_E after that
 *   clamp is SHOUJI_ERR_RANGE).  One pair per lane; no workspace.
 */
int shouji_filter_magnet(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths, int32_t E,
                         uint8_t *out_accept, int16_t *out_popcount, int64_t n_pairs, int32_t max_len,
                         int64_t ld, void *stream);

/*
 * Verifier: the aligner's threshold test for the pairs a filter accepted.
 *
 * A filtered pair goes on to alignment (Sec. 1; Sec. 3.3 and Table 3 measure
 * the filter in front of aligners).  This computes, on the GPU, the
 * unit-cost global edit distance of read and reference (equal lengths) for
 * the pairs with filter_accept[p] == 1 (every pair when filter_accept is
 * NULL), on the band |i - j| <= E (exact for the test "distance <= E": a path
 * that leaves the band has more than E indels), with the bit-vector
 * recurrence of Myers (1999) over a diagonal band of 32 rows (E <= 15) or 64
 * rows (E <= 31) per pair.
 *
 *   reads, refs, lengths, ld, max_len, n_pairs, stream: as for shouji_filter.
 *   E             threshold, 0..SHOUJI_MAX_E (else SHOUJI_ERR_ARG / _RANGE).
 *   filter_accept n_pairs bytes from a filter (device), or NULL.
 *   out_distance  n_pairs int16 (device): the distance if it is <= E, -1 if
 *                 it is larger, -2 for a pair not accepted by the filter (not
 *                 verified), -3 for a length outside [0, max_len].
 *   workspace     device buffer of shouji_verify_workspace_bytes(n_pairs)
 *                 bytes (a list of the pairs to verify), owned by the caller;
 *                 nothing is allocated.
 */
int64_t shouji_verify_workspace_bytes(int64_t n_pairs);

int shouji_verify(const uint32_t *reads, const uint32_t *refs, const int32_t *lengths, int32_t E,
                  const uint8_t *filter_accept, int16_t *out_distance, int64_t n_pairs, int32_t max_len,
                  int64_t ld, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * Serving form: a request server with continuous batching.
 *
 * Same filter (Sec. 2.2, Eq. 1, Algorithm 1) served to a stream of requests
 * of any size.  The references live in a packed pool in device memory that the
 * caller fills once (candidate locations of a read mapper point into it); a
 * request names, per pair, the offset of its reference segment in the pool.
 * The server splits its device memory budget into batch slots of
 * max_batch_pairs pairs.  Whenever a slot is free and requests are queued,
 * it takes queued pairs in arrival order (a request may span several batches
 * and a batch several requests), copies them to the device and runs the
 * batched form on them on the slot's own stream; results are copied back into
 * the request's buffers.  Each pair's result is the one shouji_filter gives
 * that pair alone, whatever else is batched with it.
 *
 * Unlike the calls above, requests are HOST buffers; the pool is a device
 * buffer.  All device and pinned host memory is allocated by
 * shouji_server_create and released by shouji_server_destroy.  Submit, poll,
 * wait and get_stats may be called from any thread.
 */
typedef struct shouji_server shouji_server;

typedef struct {
    const uint32_t *pool;    /* device: reference pool, 16 bases per word, base b in
                                bits [2*(b%16), 2*(b%16)+1] of word b/16; owned by the
                                caller and left unchanged while the server exists */
    int64_t pool_bases;      /* bases in the pool (> 0)                               */
    int32_t max_len;         /* longest pair any request holds, 1..SHOUJI_MAX_LEN     */
    int32_t slots;           /* batches in flight at most (> 0)                       */
    int64_t max_batch_pairs; /* pairs per batch slot (> 0)                            */
    int64_t memory_budget;   /* device bytes the slots may take, 0 = no limit; fewer
                                slots are made when `slots` would not fit, and
                                SHOUJI_ERR_NOMEM is returned when not even one does   */
    int32_t host_threads;    /* threads staging a batch into pinned memory (0: 8)     */
    int32_t fill_wait_us;    /* batch fill wait, 0..1000000 microseconds (0: none):
                                while another batch is in flight and fewer than
                                max_batch_pairs pairs are queued, a free slot waits
                                until this long after the oldest queued request was
                                submitted before it takes them, so that batches under
                                a steady stream run fuller; with no batch in flight a
                                slot never waits                                      */
} shouji_server_config;

typedef struct {
    const uint32_t *reads;      /* host, pair-major: read p in words
                                   [p*words_per_read, (p+1)*words_per_read), packed
                                   as the pool (base j in word j/16); with
                                   SHOUJI_REQUEST_PACKED the reads back to back
                                   instead (see there)                               */
    int32_t words_per_read;     /* > 0; words beyond ceil(max_len/16) are ignored
                                   (ignored for a packed request)                     */
    const int64_t *ref_offsets; /* host: pool base where pair p's reference begins     */
    const int32_t *lengths;     /* host: length m_p of read and reference              */
    const int32_t *E;           /* host: edit threshold of pair p                      */
    uint8_t *out_accept;        /* host: 1 accept, 0 reject, 0xFF invalid pair         */
    int16_t *out_popcount;      /* host or NULL: ones of the Shouji bit-vector, -1 for
                                   an invalid pair                                     */
    int64_t n_pairs;            /* >= 0                                                */
    uint32_t flags;             /* SHOUJI_REQUEST_* bits                               */
    int64_t read_words;         /* SHOUJI_REQUEST_PACKED: words the `reads` buffer
                                   holds; submit checks it against the lengths (see
                                   there).  Ignored for reads in rows.                */
} shouji_request;

/* The request's buffers are pinned host memory (hipHostMalloc): when its read
 * rows are ceil(max_len/16) words wide, or the reads are packed, they move by
 * DMA straight to and from the device, without a copy through the server's
 * staging buffers. */
#define SHOUJI_REQUEST_PINNED 1u

/* The reads are stored back to back with no padding: read p takes
 * ceil(m_p/16) words, none when m_p lies outside [1, max_len], and begins
 * where read p-1 ends, so `reads` holds the sum of these counts.  The server
 * moves only these words to the device (a read of m bases costs ceil(m/16)
 * words on the host link instead of ceil(max_len/16)).  The request states the
 * buffer's size in read_words; submit sums the counts from the lengths and
 * returns SHOUJI_ERR_ARG, queueing nothing, when read_words is smaller. */
#define SHOUJI_REQUEST_PACKED 2u

typedef struct {
    int32_t slots;          /* batch slots the memory budget allowed */
    int64_t batches;        /* batches launched so far               */
    int64_t pairs_done;     /* pairs whose results were delivered    */
    int64_t requests_done;  /* requests completed                    */
    int64_t requests_deferred; /* requests that found every slot busy or
                                  pairs already queued when submitted */
    int64_t queued_pairs;   /* pairs waiting for a slot              */
} shouji_server_stats;

/* Device bytes one batch slot of max_batch_pairs pairs of at most max_len bases
 * takes (to size memory_budget); negative status on bad arguments. */
int64_t shouji_server_slot_bytes(int64_t max_batch_pairs, int32_t max_len);

/* Create a server on the current device.  Invalid sizes: SHOUJI_ERR_ARG or
 * SHOUJI_ERR_RANGE; allocation failure: SHOUJI_ERR_NOMEM (nothing is leaked). */
int shouji_server_create(const shouji_server_config *config, shouji_server **out);

/* Queue a request and return its ticket.  The request's buffers are read and
 * written by the server until shouji_server_wait returns for this ticket; the
 * caller keeps them alive and untouched until then.  Submit reads the lengths
 * once (a packed request's word count is checked against them).  A pair whose length lies
 * outside [0, max_len], whose segment is not inside the pool, whose E is
 * negative or, after clamping to m-1, above SHOUJI_MAX_E gets the sentinels. */
int shouji_server_submit(shouji_server *server, const shouji_request *request, uint64_t *ticket);

/* *done = 1 when the request's results are in its buffers, else 0. */
int shouji_server_poll(shouji_server *server, uint64_t ticket, int32_t *done);

/* Block until the request is complete, return its latency (submit to results
 * delivered) in *latency_ms (may be NULL) and forget the ticket.  A device
 * failure in one of its batches is returned as SHOUJI_ERR_DEVICE. */
int shouji_server_wait(shouji_server *server, uint64_t ticket, double *latency_ms);

int shouji_server_get_stats(shouji_server *server, shouji_server_stats *stats);

/* Finish every queued request, then release all memory.  NULL is a no-op. */
int shouji_server_destroy(shouji_server *server);

/* Text of the last non-OK status returned on this thread ("" if none). */
const char *shouji_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int shouji_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHOUJI_H */
