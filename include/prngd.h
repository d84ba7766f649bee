/*
 * prngd.h -- C ABI of libprngd, an MI355X (gfx950) library that fills FP64
 * device buffers with PRNGD uniforms: Demchik & Gulov, "Increasing precision
 * of uniform pseudorandom number generators", arXiv:1401.8230.
 *
 * What one output is (Section 2 of the paper, in integer units):
 *   - A pair (x1, x2) of w-bit integers is drawn from a base generator
 *     (the paper's z = x1 + k x2 with k = 2^-w, Eq. (1)).
 *   - The pair is rejected if x1 lies in the rejection intervals
 *     x1 < a0 + k(b - b0) or x1 > a - k(b - b0) (Section 2); for integer x1
 *     with 1 <= b - b0 < 2^w these are exactly x1 = a0 and x1 = a.  By
 *     default a rejected pair consumes both words (prngd_set_consume
 *     selects Algorithm 1's one-word redraw instead).
 *   - An accepted pair is mapped by Eq. (5):
 *         N  = (x1 - a0 - 1) 2^w + (x2 - b0)         exact 64-bit integer
 *         D  = (a - a0 - 2) 2^w + (b - b0)
 *         S  = RN((1 - 2^-2w) / D)                    computed exactly once
 *         z' = RN(RN(N) * S), and z' = 1 - 2^-53 if that rounds to 1.0
 *     so z' lies in [0, 1) with z' = 0 for (a0 + 1, b0).  All roundings are
 *     IEEE round-to-nearest-even; this order of operations is part of the
 *     definition (other orders differ in the last bit).
 *   - Outputs of a stream appear in the order of their pairs.  The stream
 *     position ("pair counter") counts pairs consumed, rejected included.
 *
 * Base generators and their word layout:
 *   PRNGD_PHILOX4X32_10: Philox4x32-10 (Salmon et al., SC'11) with key
 *       (seed mod 2^32, seed / 2^32) and block counter
 *       (b mod 2^32, b / 2^32, 0, stream_id); word j is lane j mod 4 of
 *       block j / 4.  Pair p = (word 2p >> (32 - w), word 2p+1 >> (32 - w)),
 *       x1, x2 in [0, 2^w - 1], 2 <= w <= 32.
 *   PRNGD_MRG32K3A: MRG32k3a (L'Ecuyer 1999), integer outputs in
 *       [1, 4294967087].  Stream (seed, stream_id) starts from the state
 *       12345 (six times) advanced by seed * 2^127 + stream_id * 2^76 steps.
 *       Pair p = (output 2p, output 2p + 1); w = 32.
 *   PRNGD_PHILOX_X1_MRG32K3A_X2: the paper's general case of two different
 *       generators: x1 = Philox word p in [0, 2^32 - 1], x2 = MRG32k3a output
 *       p in [1, 4294967087]; w = 32.
 *   PRNGD_ENUMERATE: a test generator, pair p = ((p >> w) mod 2^w,
 *       p mod 2^w), 2 <= w <= 16; it visits every pair once per 2^2w.
 *   PRNGD_RANMAR: RANMAR (Marsaglia, Zaman, Tsang 1990, in F. James's
 *       form, Comput. Phys. Commun. 60 (1990) 329), one of the 24-bit
 *       generators Section 2 names as suitable; w = 24, words in
 *       [0, 2^24 - 1].  In units of 2^-24: L[n] = (L[n-97] - L[n-33]) mod
 *       2^24 from the 97 values of its seeds (ij, kl), C[n] = (C[n-1] -
 *       7654321) mod 16777213 from C[0] = 362436, word j = (L[j+1] -
 *       C[j+1]) mod 2^24.  Stream (seed, stream_id) is the sequence s =
 *       (seed 2^32 + stream_id) mod (31329 * 30082), ij = s / 30082,
 *       kl = s mod 30082; pair p = (word 2p, word 2p + 1).  A lagged
 *       generator: each handle keeps the 97 lagged values and C at its
 *       position on the device (about 1 KB), prngd_set_position computes
 *       them on the host (x^n mod (x^97 + x^64 - 1), about a millisecond),
 *       and a long fill starts its segments by the same jump, from a table
 *       the library builds on the host once per size.  Pair consumption,
 *       two words per output, any map; resident plans of requests of at
 *       most 32768 planned pairs; no prngd_fill_noalloc
 *       (PRNGD_ERR_UNSUPPORTED for what is not offered).
 *
 * Conventions for every call:
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Device pointers are plain device addresses owned by the caller
 *     (for example torch tensors); the library never frees them.
 *   - Calls return prngd_status_t; argument errors are detected on the
 *     host before anything is enqueued.  Work is enqueued asynchronously
 *     unless a call says it synchronises.
 *   - A handle must not be used from two host threads at once.
 *   - Errors detected on the device (a stalled cross-block scan, which a
 *     correct launch never produces) are reported by the next call on any
 *     handle as PRNGD_ERR_DEVICE.
 */
#ifndef PRNGD_H
#define PRNGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PRNGD_OK = 0,
    PRNGD_ERR_INVALID_ARGUMENT = 1,
    PRNGD_ERR_UNSUPPORTED = 2,
    PRNGD_ERR_OUT_OF_MEMORY = 3,
    PRNGD_ERR_HIP = 4,
    PRNGD_ERR_DEVICE = 5
} prngd_status_t;

typedef enum {
    PRNGD_PHILOX4X32_10 = 0,
    PRNGD_MRG32K3A = 1,
    PRNGD_PHILOX_X1_MRG32K3A_X2 = 2,
    PRNGD_ENUMERATE = 3,
    PRNGD_RANMAR = 4
} prngd_generator_t;

/* How an accepted pair becomes an output (Section 2 of the paper):
 *   PRNGD_MAP_EQ5       Eq. (5), the default: z' = RN(RN(N) * S) in [0, 1),
 *                       forced to 1 - 2^-53 if it rounds to 1 (see above).
 *   PRNGD_MAP_EQ4       Eq. (4), Algorithm 1's Z: the accepted region onto
 *                       the open interval (0, 1).  In integer units
 *                       N4 = (x1 - a0) 2^w + x2 - b = N + 2^w - (b - b0),
 *                       D4 = (a - a0) 2^w - (b - b0), S4 = RN(1 / D4),
 *                       z' = RN(RN(N4) * S4), forced below 1 the same way.
 *   PRNGD_MAP_ONE_MINUS 1 - z' of Eq. (5), one rounding: no zero, (0, 1]
 *                       (the paper's remedy where zero must not occur). */
typedef enum {
    PRNGD_MAP_EQ5 = 0,
    PRNGD_MAP_EQ4 = 1,
    PRNGD_MAP_ONE_MINUS = 2
} prngd_map_t;

/* What a rejected x1 consumes:
 *   PRNGD_CONSUME_PAIR   the whole pair (the default; Section 2's text moves
 *                        on to the following pair); the position counts
 *                        pairs.
 *   PRNGD_CONSUME_SINGLE one word, as in Algorithm 1, whose loop redraws
 *                        only r1; r2 is the word right after the accepted
 *                        r1, and the position counts words.  Streams of
 *                        one generator only: Philox (word j as above),
 *                        MRG32k3a (word j = output j) and the test generator
 *                        (words 2p, 2p + 1 = pair p's x1, x2);
 *                        PRNGD_ERR_UNSUPPORTED for the mixed generator.
 *                        A batch produces each request in one workgroup; a
 *                        single prngd_fill of at least 2^15 outputs that
 *                        expects at most 64 words equal to a0 or a (256 when
 *                        a speculative path is forced by prngd_set_tuning)
 *                        spreads its windows of 4096 words over
 *                        workgroups and repairs them in a second kernel on
 *                        the same stream. */
typedef enum {
    PRNGD_CONSUME_PAIR = 0,
    PRNGD_CONSUME_SINGLE = 1
} prngd_consume_t;

typedef struct prngd_handle_s *prngd_handle_t;
typedef struct prngd_plan_s *prngd_plan_t;

/* One fill request of a batch: the next n outputs of handle h into out. */
typedef struct {
    prngd_handle_t h;
    uint64_t n;
    double *out;
} prngd_request_t;

/* Launch shape of the fill kernels.  None of these change the output
 * bytes; they only change speed.  Zero fields mean "library default". */
typedef struct {
    uint32_t pairs_per_lane;  /* pairs per thread per tile: 2, 4, 8, 16, 32 */
                              /* (0: 8 for a single Philox fill that takes  */
                              /* path 2 or 3, 16 otherwise)                 */
    uint32_t blocks_per_cu;   /* workgroups per CU (0: all that fit)        */
    uint32_t store_mode;      /* 0 default, 1 plain 8-byte, 2 nontemporal   */
    uint32_t slack_mode;      /* 0 plan rejections ahead, 1 plan none (the  */
                              /* last tile then absorbs every rejection)    */
    uint32_t block_threads;   /* threads per workgroup: 256, 512, 1024      */
    uint32_t seq_max_tiles;   /* batch requests of at most this many tiles  */
                              /* are produced whole by one workgroup; the   */
                              /* rest are split over workgroups joined by   */
                              /* the look-back (0: half a fair share)       */
    uint32_t path;            /* 0 automatic; 1 ordered (look-back and      */
                              /* segment-sequential kernels); 2 speculative */
                              /* (each tile stores at the offset it assumes */
                              /* from the rejections published so far, a    */
                              /* repair pass redoes tiles that assumed      */
                              /* wrong); 3 speculative, holding the window  */
                              /* in registers until its offset is read;     */
                              /* 4 speculative in 128-pair chunks, one per  */
                              /* wave, for single fills (batches take 2);   */
                              /* 5 as 4, and batches in chunks of           */
                              /* pairs_per_lane / 2 windows of 128 pairs    */
                              /* (1, 2 or 4), one per wave: every chunk     */
                              /* of every request stores                    */
                              /* at the offset no earlier rejection gives,  */
                              /* a repair pass redoes each request from its */
                              /* first chunk with a rejection (Philox and   */
                              /* the test generator; others take 2);        */
                              /* 6 counted, for single fills of Philox or   */
                              /* the test generator: one kernel counts the  */
                              /* accepted pairs of every 512-pair chunk, a  */
                              /* scan turns counts into offsets, a second   */
                              /* kernel produces every chunk at its offset  */
                              /* (nothing is redone; at most 2^31 pairs;    */
                              /* other fills as automatic).                 */
                              /* Automatic: 6 for a single fill of Philox   */
                              /* or the test generator of at least 2^18     */
                              /* pairs that expects more than 2             */
                              /* rejections; 5 for a batch of Philox or     */
                              /* test generator requests of at most 2^16    */
                              /* pairs                                      */
                              /* that expects at most 256 rejections;       */
                              /* otherwise ordered unless some request has  */
                              /* at least 2^18 pairs; then, single fills: 3 */
                              /* at w = 32 up to 2 expected rejections, 4   */
                              /* up to 1024; batches: 3 up to 128.          */
                              /* MRG32k3a and mixed have form 3 only        */
} prngd_tuning_t;

/* Human-readable name of a status code (static storage). */
const char *prngd_status_string(prngd_status_t status);

/* Message of the last error returned to this host thread ("" if none). */
const char *prngd_last_error(void);

/*
 * Validate (generator, k, min, max) and return the constants of Eq. (5)
 * without touching a GPU.  Algorithm 1 of the paper is PRNGD(k, min, max):
 * k must be exactly 2^-w, and [min, max] must be the extreme values the
 * generator's x1 can take (its natural range for that w): Philox and
 * ENUMERATE [0, 2^w - 1], MRG32k3a [1, 4294967087], mixed [0, 2^32 - 1].
 * Any output pointer may be NULL.
 * Errors: PRNGD_ERR_INVALID_ARGUMENT (k not a power 2^-w, w out of range
 * for the generator, range mismatch), PRNGD_ERR_UNSUPPORTED (unknown
 * generator).
 */
prngd_status_t prngd_describe(prngd_generator_t generator, double k,
                              uint64_t min, uint64_t max, uint32_t *w,
                              uint64_t *b0, uint64_t *b, uint64_t *D,
                              double *S);

/*
 * The constants of one map for (generator, k, min, max), host only: the
 * offset added to N (2^w - (b - b0) for Eq. (4), else 0), the denominator
 * (D, or D4 for Eq. (4)) and the folded constant S.  Any output pointer
 * may be NULL.  Errors: as prngd_describe; PRNGD_ERR_INVALID_ARGUMENT for
 * an unknown map.
 */
prngd_status_t prngd_describe_map(prngd_generator_t generator, double k,
                                  uint64_t min, uint64_t max, prngd_map_t map,
                                  uint64_t *n_offset, uint64_t *D, double *S);

/*
 * Create a PRNGD stream handle on the current HIP device: Algorithm 1's
 * PRNGD(k, min, max) with a base generator and a seed.  Stream id 0, pair
 * counter 0.  The library allocates the handle and its device state (two
 * 64-bit counters) and owns both until prngd_destroy.
 * Errors: as prngd_describe; PRNGD_ERR_INVALID_ARGUMENT for a NULL
 * out_handle; PRNGD_ERR_OUT_OF_MEMORY; PRNGD_ERR_HIP.
 */
prngd_status_t prngd_create(uint64_t seed, prngd_generator_t generator,
                            double k, uint64_t min, uint64_t max,
                            prngd_handle_t *out_handle);

/*
 * Create `count` handles on the consecutive substreams first_stream_id,
 * first_stream_id + 1, ... of one seed, all at pair counter 0 -- the
 * independent streams of a Monte Carlo run.  Equivalent to prngd_create
 * followed by prngd_set_position(h, first_stream_id + i, 0) for each, but
 * enqueues no GPU work.  On error no handle is left allocated.
 * Errors: as prngd_create; PRNGD_ERR_INVALID_ARGUMENT for a NULL handles
 * array or substream ids beyond 2^32 - 1.
 */
prngd_status_t prngd_create_many(uint64_t seed, prngd_generator_t generator,
                                 double k, uint64_t min, uint64_t max,
                                 uint32_t first_stream_id, uint32_t count,
                                 prngd_handle_t *handles);

/*
 * RANMAR state of stream (seed, stream_id) of PRNGD_RANMAR at pair
 * position pair_counter (word 2 pair_counter), host only:
 * out[0 .. 96] = L[W - 96 .. W] and out[97] = C[W] in units of 2^-24
 * (W = 2 pair_counter; see PRNGD_RANMAR above), the values a handle keeps
 * on the device there.  Errors: PRNGD_ERR_INVALID_ARGUMENT for a NULL out.
 */
prngd_status_t prngd_ranmar_state(uint64_t seed, uint32_t stream_id, uint64_t pair_counter,
                                  uint32_t out[98]);

/* Choose the map of the handle's later outputs (PRNGD_MAP_EQ5 after
 * prngd_create).  Host only; fills already enqueued are not affected.
 * Handles of one batch must share their map.  Errors:
 * PRNGD_ERR_INVALID_ARGUMENT (NULL handle, unknown map, handle bound to a
 * live plan). */
prngd_status_t prngd_set_map(prngd_handle_t h, prngd_map_t map);
prngd_status_t prngd_get_map(prngd_handle_t h, prngd_map_t *map);

/* Choose what a rejection consumes for the handle's later fills
 * (PRNGD_CONSUME_PAIR after prngd_create).  The position is not converted:
 * it counts pairs in one mode and words in the other.  Handles of one
 * batch must share it.  Errors: PRNGD_ERR_INVALID_ARGUMENT (NULL handle,
 * unknown mode, handle bound to a live plan), PRNGD_ERR_UNSUPPORTED. */
prngd_status_t prngd_set_consume(prngd_handle_t h, prngd_consume_t consume);
prngd_status_t prngd_get_consume(prngd_handle_t h, prngd_consume_t *consume);

/*
 * Words combined per output: 2 (Section 2, after prngd_create) or 3, the
 * generalisation the paper's Conclusion names (more than two PRNs for a
 * greater precision), read as the two-word method applied twice:
 *   - triple t is words 3t, 3t + 1, 3t + 2 of the stream;
 *   - the inner pair (x2, x3) is accepted by Section 2's rule into
 *     y = x2 + k x3, of resolution k^2; the outer pair (x1, y) by the same
 *     rule with y's span in place of b - b0.  Both reduce to x1 and x2 not
 *     in {a0, a}; a rejection at either level consumes the whole triple;
 *   - Eq. (5) maps z = x1 + k y with k' = k^3; in integer units
 *     N3 = (x1 - a0 - 1) 2^2w + (x2 - a0 - 1) 2^w + (x3 - a0),
 *     D3 = (a - a0 - 2) 2^2w + (a - a0 - 2) 2^w + (a - a0),
 *     S3 = RN((1 - 2^-3w) / D3) computed exactly on the host, and
 *     z' = RN(RN(N3) * S3) with RN(N3) the correctly rounded value of the
 *     exact integer (3w bits: exact in FP64 up to w = 17), forced to
 *     1 - 2^-53 if it rounds to 1.
 * The position then counts triples (prngd_set_position's pair_counter is a
 * triple counter; it is not converted).  Philox4x32-10 (any w) and the test
 * generator only, with PRNGD_MAP_EQ5 and PRNGD_CONSUME_PAIR; such handles
 * fill through the ordered kernels in batches and plans, and a single fill
 * of at least 16384 triples counts the kept triples of every 4096-triple
 * window, scans the counts and produces every window at its offset (path 1
 * of prngd_set_tuning keeps the ordered kernels).  Handles of
 * one batch must share it.  Errors: PRNGD_ERR_INVALID_ARGUMENT (NULL
 * handle, words not 2 or 3, handle bound to a live plan),
 * PRNGD_ERR_UNSUPPORTED (another generator, map or consumption; setting a
 * map or consumption other than the defaults on a three-word handle).
 */
prngd_status_t prngd_set_arity(prngd_handle_t h, uint32_t words);
prngd_status_t prngd_get_arity(prngd_handle_t h, uint32_t *words);

/* Wait for the handle's outstanding work, then free it.  NULL is a no-op. */
prngd_status_t prngd_destroy(prngd_handle_t h);

/*
 * Move the handle to (stream_id, pair_counter): the next fill starts with
 * pair pair_counter of substream stream_id (Philox counter word 3; MRG32k3a
 * jump of stream_id * 2^76).  Enqueued on `stream` after the handle's
 * previous work.  Errors: PRNGD_ERR_INVALID_ARGUMENT (NULL handle, handle
 * bound to a live plan), PRNGD_ERR_HIP.
 */
prngd_status_t prngd_set_position(prngd_handle_t h, uint32_t stream_id,
                                  uint64_t pair_counter, void *stream);

/*
 * Read the handle's position (a checkpoint: a new handle with the same
 * seed, generator and position continues the same sequence).
 * SYNCHRONISES `stream` after the handle's previous work.
 */
prngd_status_t prngd_get_position(prngd_handle_t h, uint32_t *stream_id,
                                  uint64_t *pair_counter, void *stream);

/*
 * out[0 .. n) = the next n outputs of the handle, in sequential order, and
 * the handle's pair counter advances past the pair of out[n - 1].
 * `out` is caller-owned device memory, 8-byte aligned, at least 8n bytes.
 * n = 0 is a no-op.  Asynchronous on `stream`; fills of one handle are
 * ordered (a fill on a different stream first waits for the handle's
 * previous work).  Errors: PRNGD_ERR_INVALID_ARGUMENT (NULL handle, NULL or
 * misaligned out with n > 0, handle bound to a live plan), PRNGD_ERR_HIP,
 * PRNGD_ERR_DEVICE.
 */
prngd_status_t prngd_fill(prngd_handle_t h, uint64_t n, double *out,
                          void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * output and the same new position as prngd_fill, from a variant that
 * allocates nothing.  Its launch state (the look-back kernel's ticket
 * counter and one 8-byte status word per tile) lives in a fixed 4 MiB
 * device array that each GPU holds until the process ends, set up when the
 * library first meets the device (prngd_create); so n is limited to
 * 524224 tiles of the handle's launch shape (threads x pairs per lane
 * pairs, 4096 by default: about 2.1e9 outputs).  Every call on one GPU
 * shares that array and finds it as the previous call left it: calls on
 * one GPU must not overlap -- issue them on one stream, or order them
 * yourself; calls that overlap race.  Pair consumption only.  MRG32k3a
 * and mixed handles use the jump tables built when they were created (for
 * the launch shape set then).  Errors: as prngd_fill, plus
 * PRNGD_ERR_INVALID_ARGUMENT when n needs more tiles than the array holds,
 * PRNGD_ERR_UNSUPPORTED for one-word consumption or a launch shape whose
 * MRG32k3a tables do not exist yet.
 */
prngd_status_t prngd_fill_noalloc(prngd_handle_t h, uint64_t n, double *out,
                                  void *stream);

/*
 * Fill several handles in one persistent launch: request i receives
 * exactly what prngd_fill(reqs[i].h, reqs[i].n, reqs[i].out) would give,
 * bit for bit, and each handle advances as it would.  `reqs` is read
 * before the call returns.  All handles must be distinct and share the
 * generator, k, min, max, map and consumption; requests with n = 0 are
 * skipped.
 * Errors: PRNGD_ERR_INVALID_ARGUMENT (count = 0 with reqs NULL, a NULL or
 * repeated handle, mixed configurations, bad out), PRNGD_ERR_HIP.
 */
prngd_status_t prngd_fill_batch(const prngd_request_t *reqs, uint32_t count,
                                void *stream);

/*
 * A resident batch: the request descriptors are uploaded once and the
 * persistent fill kernel is captured in a HIP graph.  Each
 * prngd_plan_launch replays the graph and is equivalent to
 * prngd_fill_batch(reqs, count) with the handles' positions at that
 * moment.  While the plan lives, its handles may only be advanced through
 * it (other fills on them return PRNGD_ERR_INVALID_ARGUMENT).  A plan must
 * not be launched concurrently with itself.
 */
prngd_status_t prngd_plan_create(const prngd_request_t *reqs, uint32_t count,
                                 prngd_plan_t *out_plan);
prngd_status_t prngd_plan_launch(prngd_plan_t plan, void *stream);
prngd_status_t prngd_plan_destroy(prngd_plan_t plan);

/* Process-wide launch shape for one (generator, w); tuning never changes
 * output bytes.  prngd_get_tuning returns the shape in effect. */
prngd_status_t prngd_set_tuning(prngd_generator_t generator, uint32_t w,
                                const prngd_tuning_t *tuning);
prngd_status_t prngd_get_tuning(prngd_generator_t generator, uint32_t w,
                                prngd_tuning_t *tuning);

#ifdef __cplusplus
}
#endif
#endif /* PRNGD_H */
