/*
 * prngd_oracle.h -- CPU oracle for the PRNGD method.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential, obviously
 * checkable CPU implementation of what the PRNGD fill computes, written from
 * Demchik & Gulov, "Increasing precision of uniform pseudorandom number
 * generators" (arXiv:1401.8230), Section 2 and Algorithm 1.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Parity status of each part (what pins it is listed in the tests):
 *   - RANMAR: pinned by the check values its published description gives
 *     (seeds 1802, 9373: words 20000 .. 20005), and jump == stepping.
 *   - Philox4x32-10 block function: pinned against an independent library
 *     implementation (rocRAND, built from its source headers for the host)
 *     and by counter-carry / split invariants.
 *   - MRG32k3a: pinned by stepping == matrix jump-ahead, by the full-period
 *     identity A^(m^3-1) == I for both components, and against rocRAND.
 *   - Accept/reject (Section 2, rejection intervals and the discrete
 *     degeneration to x1 in {a0, a}): exhaustive enumeration at w = 8,
 *     rejection fraction exactly 2/2^w, brute-force interval checks.
 *   - Affine map, Eq. (5)/(6): endpoints, closed form within the rounding
 *     bound (exact rationals), each grid value exactly once at w = 8.
 *
 * Conventions that the paper leaves open (the readings are stated here and
 * in the design notes):
 *   - Generator words are unsigned integers; the paper's w-bit PRN x in
 *     [0, 1) with step k = 2^-w is the integer X = x / k.  All formulas below
 *     are the paper's formulas scaled by 2^w, which changes no ratio.
 *   - A rejected pair consumes both of its words (Section 2's text).
 *   - The constant part of Eq. (5) is folded into one FP64 constant
 *     S = RN((1 - k^2) / D); the output is RN(RN(N) * S), clamped below 1.
 */
#ifndef PRNGD_ORACLE_H
#define PRNGD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Base generators known to the oracle. */
enum {
    ORC_GEN_PHILOX    = 0, /* pair p = (word 2p, word 2p+1) >> (32 - w)       */
    ORC_GEN_MRG32K3A  = 1, /* pair p = (output 2p, output 2p+1), w = 32       */
    ORC_GEN_MIXED     = 2, /* pair p = (Philox word p, MRG32k3a output p)      */
    ORC_GEN_ENUMERATE = 3, /* pair p = ((p >> w) mod 2^w, p mod 2^w), tests    */
    ORC_GEN_RANMAR    = 4  /* pair p = (RANMAR word 2p, word 2p+1), w = 24     */
};

/* How an accepted pair becomes an output (Section 2). */
enum {
    ORC_MAP_EQ5       = 0, /* Eq. (5): z' in [0, 1), the default              */
    ORC_MAP_EQ4       = 1, /* Eq. (4), Algorithm 1's Z: z' in (0, 1)          */
    ORC_MAP_ONE_MINUS = 2  /* 1 - z' of Eq. (5): no zero, in (0, 1]           */
};

/* What a rejected x1 consumes. */
enum {
    ORC_CONSUME_PAIR   = 0, /* the whole pair (the text of Section 2)        */
    ORC_CONSUME_SINGLE = 1  /* one word (Algorithm 1: only r1 is redrawn);
                               single-generator streams only               */
};

/* One PRNGD stream: which generator, the ranges of x1 and x2 (integer
 * units), and the position (pairs consumed so far, rejected ones included). */
typedef struct {
    int      generator;
    int      w;        /* resolution k = 2^-w                          */
    uint64_t seed;
    uint32_t stream;
    uint64_t counter;  /* pairs consumed (words, when consume = single) */
    uint64_t a0, a;    /* x1 in [a0, a]                                */
    uint64_t b0, b;    /* x2 in [b0, b]                                */
    uint64_t D;        /* (a - a0 - 2) * 2^w + (b - b0)                */
    double   S;        /* RN((1 - 2^-2w) / D)                          */
    int      map;      /* ORC_MAP_*                                     */
    uint64_t D4;       /* Eq. (4) in integer units: (a - a0) 2^w - (b - b0) */
    double   S4;       /* RN(1 / D4)                                    */
    int      consume;  /* ORC_CONSUME_*                                 */
    uint32_t mrg[6];   /* MRG32k3a state at stream position 0          */
    int      arity;    /* words per output: 2, or 3 (orc_set_arity)     */
    uint64_t D3_hi;    /* three words: D3 = (a - a0 - 2) 2^2w + Y1 - Y0 */
    uint64_t D3_lo;    /*   (a 128-bit integer, two halves)             */
    double   S3;       /* RN((1 - 2^-3w) / D3)                          */
    uint32_t ranmar[97]; /* RANMAR lagged values L[-96..0] of the stream  */
} orc_stream;

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
/* Words [first, first + count) of the Philox stream (seed, stream):
 * word j is lane j mod 4 of block j / 4, block b has counter
 * (b mod 2^32, b / 2^32, 0, stream) and key (seed mod 2^32, seed / 2^32). */
void orc_philox_words(uint64_t seed, uint32_t stream, uint64_t first,
                      uint64_t count, uint32_t *out);

/* ---- MRG32k3a (L'Ecuyer, Operations Research 47(1), 1999) ------------- */
/* state: (s10, s11, s12, s20, s21, s22); exponent: little-endian 64-bit
 * limbs, nlimbs <= 3. */
void orc_mrg_jump(uint32_t state[6], const uint64_t *exponent, int nlimbs);
void orc_mrg_outputs(uint32_t state[6], uint64_t count, uint32_t *out);
void orc_mrg_matpow(int component, const uint64_t *exponent, int nlimbs,
                    uint64_t out[9]);
/* State at position 0 of stream (seed, stream): the six-fold 12345 state
 * advanced by seed * 2^127 + stream * 2^76 steps. */
void orc_mrg_stream_base(uint64_t seed, uint32_t stream, uint32_t out[6]);

/* ---- RANMAR (Marsaglia, Zaman, Tsang, Stat. Prob. Lett. 9 (1990) 35;
 * F. James, Comput. Phys. Commun. 60 (1990) 329) ------------------------
 * In integer units of 2^-24.  Lagged values L[n] = (L[n-97] - L[n-33])
 * mod 2^24 for n >= 1 from 97 seed values L[-96..0]; an arithmetic part
 * C[n] = (C[n-1] - 7654321) mod 16777213, C[0] = 362436; word j of the
 * stream (j = 0, 1, ...) is (L[j+1] - C[j+1]) mod 2^24.  The seed values
 * come from the generator's two seeds ij in [0, 31328], kl in [0, 30081]
 * (a lagged Fibonacci and a congruential generator, 24 bits each); a
 * PRNGD stream (seed, stream) uses sequence s = (seed 2^32 + stream) mod
 * (31329 * 30082), ij = s / 30082, kl = s mod 30082.
 * A "window" at word position n is L[n-96 .. n] (window[i] = L[n-96+i])
 * with C[n]; the next word is made from window[0] - window[64]. */
void orc_ranmar_seed(uint32_t ij, uint32_t kl, uint32_t window[97]);
void orc_ranmar_stream_seeds(uint64_t seed, uint32_t stream, uint32_t *ij,
                             uint32_t *kl);
/* The window at word position n by stepping n times (O(n)). */
void orc_ranmar_step_to(const uint32_t window0[97], uint64_t n,
                        uint32_t window[97], uint32_t *C);
/* The same by the jump polynomial x^n mod (x^97 + x^64 - 1) over the
 * integers mod 2^24 (O(97^2 log n)). */
void orc_ranmar_jump(const uint32_t window0[97], uint64_t n_lo, uint64_t n_hi,
                     uint32_t window[97], uint32_t *C);
/* Words [first, first + count) of the sequence with seed window window0. */
void orc_ranmar_words(const uint32_t window0[97], uint64_t first,
                      uint64_t count, uint32_t *out);

/* ---- PRNGD ------------------------------------------------------------- */
/* 0 on success, -1 on invalid parameters. */
int orc_init(orc_stream *s, int generator, int w, uint64_t seed,
             uint32_t stream, uint64_t counter);
/* A stream with explicit ranges and no generator (pairs are supplied by
 * the caller to orc_accept / orc_map). */
int orc_init_ranges(orc_stream *s, int w, uint64_t a0, uint64_t a,
                    uint64_t b0, uint64_t b);
void orc_pair(const orc_stream *s, uint64_t p, uint64_t *x1, uint64_t *x2);
int orc_accept(const orc_stream *s, uint64_t x1);
double orc_map(const orc_stream *s, uint64_t x1, uint64_t x2);
/* The next n outputs of the stream, in order; advances s->counter.
 * accepted_index, if not NULL, receives the pair index of each output. */
void orc_fill(orc_stream *s, uint64_t n, double *out,
              uint64_t *accepted_index);
/* The outputs of the accepted pairs among pairs [s->counter, pair_end), in
 * order, at most max_out of them; returns how many were written and leaves
 * s->counter at the first pair not examined (triples, for three words per
 * output).  Pair consumption only (returns 0 otherwise).  Concatenating the outputs of consecutive pair ranges gives
 * orc_fill's sequence, so one long stream can be walked in pieces. */
uint64_t orc_fill_pairs(orc_stream *s, uint64_t pair_end, uint64_t max_out,
                        double *out);
/* Exact RN((2^2w - 1) / (D * 2^2w)), the folded constant of Eq. (5). */
double orc_scale(int w, uint64_t D);
/* Exact RN(1 / D), the folded constant of Eq. (4). */
double orc_recip(uint64_t D);
/* Choose the map of the stream's outputs; 0 on success, -1 if unknown. */
int orc_set_map(orc_stream *s, int map);
/* Choose what a rejection consumes; 0 on success, -1 if unknown or if the
 * stream combines two generators.  The counter then counts words. */
int orc_set_consume(orc_stream *s, int consume);
/* Word j of a single-generator stream: Philox word j >> (32 - w); MRG32k3a
 * output j; ENUMERATE: x1 of pair j / 2 for even j, x2 for odd j (with three
 * words per output: word 3t + i is digit 2 - i, base 2^w, of t). */
uint64_t orc_word(const orc_stream *s, uint64_t j);

/* ---- Three words per output (the paper's Conclusion) --------------------
 * The two-word method applied twice.  The inner pair (x2, x3) is accepted
 * by Section 2's rule and gives y = x2 + k x3, a PRN of resolution k^2 on
 * [b0', b'] = [(a0 + 1) + k a0, (a - 1) + k a] (in units of the words).
 * The outer pair (x1, y) is accepted by the same rule with b' - b0' in
 * place of b - b0, and Eq. (5) maps z = x1 + k y with k' = k^3.  In
 * integer units (all multiplied by 2^2w): Y = x2 2^w + x3,
 * Y0 = (a0 + 1) 2^w + a0, Y1 = (a - 1) 2^w + a,
 * N3 = (x1 - a0 - 1) 2^2w + (Y - Y0), D3 = (a - a0 - 2) 2^2w + (Y1 - Y0),
 * z' = RN(RN(N3) * S3), S3 = RN((2^3w - 1) / (D3 2^3w)), forced below 1
 * like the two-word map.  RN(N3) is the correctly rounded value of the
 * exact integer.  Triple t is words 3t, 3t + 1, 3t + 2; a rejection at
 * either level consumes the whole triple, and the counter counts triples.
 * Single-generator streams (Philox, MRG32k3a, ENUMERATE), Eq. (5), pair
 * consumption. */
int orc_set_arity(orc_stream *s, int arity);
/* The outer and inner acceptance tests of a triple, exact integers. */
int orc_accept3(const orc_stream *s, uint64_t x1, uint64_t x2);
double orc_map3(const orc_stream *s, uint64_t x1, uint64_t x2, uint64_t x3);
/* RN of the 128-bit integer hi 2^64 + lo (round half to even). */
double orc_rn_u128(uint64_t hi, uint64_t lo);
/* RN((2^3w - 1) / (D 2^3w)) for the 128-bit D = hi 2^64 + lo, 0 < D < 2^3w. */
double orc_scale3(int w, uint64_t D_hi, uint64_t D_lo);

#ifdef __cplusplus
}
#endif
#endif
