/*
 * prngd_oracle.c -- CPU oracle for the PRNGD method (test infrastructure).
 *
 * Plain sequential C, one stream at a time.  Every function cites the part
 * of the paper (Demchik & Gulov, arXiv:1401.8230) or the published
 * generator definition it follows.  Build: gcc -O2 -ffp-contract=off, SSE2
 * double arithmetic, round-to-nearest-even, no FMA.
 */
#include "prngd_oracle.h"

#include <math.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

/* ======================================================================
 * Philox4x32-10.  Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11, Section 3: each round multiplies counter
 * words 0 and 2 by the two Philox multipliers, keeps both halves of the
 * 64-bit products, and XORs the high halves with the other two counter
 * words and the round key; the key is bumped by the two Weyl constants
 * (golden ratio and sqrt(3) - 1, scaled to 32 bits) between rounds.
 * ====================================================================== */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {           /* key schedule: bump before rounds 2..10 */
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Lane `lane` of block `block` of the Philox stream (seed, stream): the
 * counter is (block mod 2^32, block / 2^32, 0, stream), the key is
 * (seed mod 2^32, seed / 2^32).  Word j of the stream is lane j mod 4 of
 * block j / 4. */
static uint32_t philox_lane(uint64_t seed, uint32_t stream, uint64_t block,
                            unsigned lane)
{
    uint32_t ctr[4] = { (uint32_t)block, (uint32_t)(block >> 32), 0u, stream };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    return r[lane];
}

static uint32_t philox_word(uint64_t seed, uint32_t stream, uint64_t j)
{
    return philox_lane(seed, stream, j / 4, (unsigned)(j % 4));
}

void orc_philox_words(uint64_t seed, uint32_t stream, uint64_t first,
                      uint64_t count, uint32_t *out)
{
    for (uint64_t i = 0; i < count; i++)
        out[i] = philox_word(seed, stream, first + i);
}

/* ======================================================================
 * MRG32k3a.  L'Ecuyer, "Good parameters and implementations for combined
 * multiple recursive random number generators", Oper. Res. 47(1), 1999:
 *   x1[n] = (1403580 x1[n-2] -  810728 x1[n-3]) mod m1,  m1 = 2^32 - 209
 *   x2[n] = ( 527612 x2[n-1] - 1370589 x2[n-3]) mod m2,  m2 = 2^32 - 22853
 * with integer output (x1[n] - x2[n]) mod m1, where 0 is reported as m1,
 * so outputs lie in [1, m1].  Streams and substreams follow L'Ecuyer,
 * Simard, Chen, Kelton, "An object-oriented random-number package with
 * many long streams and substreams", Oper. Res. 50(6), 2002: streams are
 * 2^127 steps apart, substreams 2^76, the package seed is 12345 six times.
 * ====================================================================== */
#define ORC_M1 4294967087ull
#define ORC_M2 4294944443ull

/* One step of the two recurrences, written directly from the definition;
 * state = (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1]). */
static uint32_t mrg_step(uint32_t st[6])
{
    uint64_t t1 = (1403580ull * st[1]) % ORC_M1;
    uint64_t u1 = (810728ull * st[0]) % ORC_M1;
    uint64_t n1 = (t1 + ORC_M1 - u1) % ORC_M1;
    uint64_t t2 = (527612ull * st[5]) % ORC_M2;
    uint64_t u2 = (1370589ull * st[3]) % ORC_M2;
    uint64_t n2 = (t2 + ORC_M2 - u2) % ORC_M2;
    st[0] = st[1]; st[1] = st[2]; st[2] = (uint32_t)n1;
    st[3] = st[4]; st[4] = st[5]; st[5] = (uint32_t)n2;
    return n1 > n2 ? (uint32_t)(n1 - n2) : (uint32_t)(n1 + ORC_M1 - n2);
}

void orc_mrg_outputs(uint32_t state[6], uint64_t count, uint32_t *out)
{
    for (uint64_t i = 0; i < count; i++)
        out[i] = mrg_step(state);
}

/* The one-step transition matrices acting on the column (x[n-3], x[n-2],
 * x[n-1]) of each component, entries reduced into [0, m). */
static void mrg_matrix(int component, uint64_t A[9])
{
    uint64_t m = component == 0 ? ORC_M1 : ORC_M2;
    memset(A, 0, 9 * sizeof(uint64_t));
    A[1] = 1;                                   /* row 0: x[n-2]          */
    A[5] = 1;                                   /* row 1: x[n-1]          */
    if (component == 0) {                       /* row 2: the recurrence  */
        A[6] = m - 810728ull;
        A[7] = 1403580ull;
        A[8] = 0;
    } else {
        A[6] = m - 1370589ull;
        A[7] = 0;
        A[8] = 527612ull;
    }
}

static void matmul_mod(const uint64_t X[9], const uint64_t Y[9], uint64_t m,
                       uint64_t Z[9])
{
    uint64_t R[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            u128 acc = 0;
            for (int l = 0; l < 3; l++)
                acc += (u128)X[3 * i + l] * Y[3 * l + j];
            R[3 * i + j] = (uint64_t)(acc % m);
        }
    memcpy(Z, R, sizeof R);
}

/* A^e mod m by square-and-multiply over the limbs of e. */
void orc_mrg_matpow(int component, const uint64_t *exponent, int nlimbs,
                    uint64_t out[9])
{
    uint64_t m = component == 0 ? ORC_M1 : ORC_M2;
    uint64_t P[9], R[9] = { 1, 0, 0, 0, 1, 0, 0, 0, 1 };
    mrg_matrix(component, P);
    for (int limb = 0; limb < nlimbs; limb++)
        for (int bit = 0; bit < 64; bit++) {
            if ((exponent[limb] >> bit) & 1u)
                matmul_mod(R, P, m, R);
            matmul_mod(P, P, m, P);
        }
    memcpy(out, R, sizeof R);
}

void orc_mrg_jump(uint32_t state[6], const uint64_t *exponent, int nlimbs)
{
    for (int c = 0; c < 2; c++) {
        uint64_t M[9], m = c == 0 ? ORC_M1 : ORC_M2;
        orc_mrg_matpow(c, exponent, nlimbs, M);
        uint32_t *v = state + 3 * c;
        uint64_t r[3];
        for (int i = 0; i < 3; i++) {
            u128 acc = 0;
            for (int l = 0; l < 3; l++)
                acc += (u128)M[3 * i + l] * v[l];
            r[i] = (uint64_t)(acc % m);
        }
        for (int i = 0; i < 3; i++)
            v[i] = (uint32_t)r[i];
    }
}

void orc_mrg_stream_base(uint64_t seed, uint32_t stream, uint32_t out[6])
{
    /* exponent seed * 2^127 + stream * 2^76 as three 64-bit limbs */
    uint64_t e[3];
    e[0] = 0;
    e[1] = ((uint64_t)stream << 12) | ((seed & 1u) << 63);
    e[2] = seed >> 1;
    for (int i = 0; i < 6; i++)
        out[i] = 12345u;
    orc_mrg_jump(out, e, 3);
}

/* ======================================================================
 * RANMAR.  Marsaglia, Zaman, Tsang, "Toward a universal random number
 * generator", Stat. Prob. Lett. 9 (1990) 35, in the form F. James gives
 * (Comput. Phys. Commun. 60 (1990) 329): a lagged Fibonacci generator
 * with lags 97 and 33 under subtraction mod 1, minus an arithmetic
 * sequence mod 16777213/16777216, all values multiples of 2^-24.  Here in
 * integer units of 2^-24 (the header states the sequence).
 * ====================================================================== */
#define ORC_RANMAR_MASK 0xFFFFFFu
#define ORC_RANMAR_CD   7654321u
#define ORC_RANMAR_CM   16777213u
#define ORC_RANMAR_C0   362436u
#define ORC_RANMAR_IJ   31329u
#define ORC_RANMAR_KL   30082u

/* The 97 seed values: four small generators (a lagged Fibonacci generator
 * on three values mod 179 and a congruential one mod 169) give one bit
 * each step, 24 steps per value, most significant bit first.  The values
 * come out for L[0], L[-1], ..., L[-96] in that order. */
void orc_ranmar_seed(uint32_t ij, uint32_t kl, uint32_t window[97])
{
    uint32_t i = (ij / 177) % 177 + 2;
    uint32_t j = ij % 177 + 2;
    uint32_t k = (kl / 169) % 178 + 1;
    uint32_t l = kl % 169;
    for (int v = 0; v < 97; v++) {
        uint32_t value = 0;
        for (int bit = 0; bit < 24; bit++) {
            uint32_t m = (((i * j) % 179) * k) % 179;
            i = j;
            j = k;
            k = m;
            l = (53 * l + 1) % 169;
            value = 2 * value + ((l * m) % 64 >= 32 ? 1u : 0u);
        }
        window[96 - v] = value;       /* value v is L[-v] */
    }
}

void orc_ranmar_stream_seeds(uint64_t seed, uint32_t stream, uint32_t *ij,
                             uint32_t *kl)
{
    u128 s = (((u128)seed << 32) | stream) % ((u128)ORC_RANMAR_IJ * ORC_RANMAR_KL);
    *ij = (uint32_t)(s / ORC_RANMAR_KL);
    *kl = (uint32_t)(s % ORC_RANMAR_KL);
}

/* C[n] = (C[0] - n * 7654321) mod 16777213, n = n_hi 2^64 + n_lo. */
static uint32_t ranmar_c_at(uint64_t n_lo, uint64_t n_hi)
{
    u128 n = ((u128)n_hi << 64) | n_lo;
    uint64_t t = (uint64_t)(n % ORC_RANMAR_CM) * ORC_RANMAR_CD % ORC_RANMAR_CM;
    return (uint32_t)((ORC_RANMAR_C0 + ORC_RANMAR_CM - t) % ORC_RANMAR_CM);
}

/* A stepping generator: the window as a ring (slot (head + i) mod 97 holds
 * window[i]) and C. */
typedef struct {
    uint32_t L[97];
    unsigned head;
    uint32_t C;
} ranmar_cursor;

static void ranmar_cursor_set(ranmar_cursor *g, const uint32_t window[97], uint32_t C)
{
    memcpy(g->L, window, sizeof g->L);
    g->head = 0;
    g->C = C;
}

/* The next word: L[n+1] = L[n-96] - L[n-32] replaces L[n-96]. */
static uint32_t ranmar_next(ranmar_cursor *g)
{
    uint32_t oldest = g->L[g->head];
    uint32_t lag33 = g->L[(g->head + 64) % 97];
    uint32_t v = (oldest - lag33) & ORC_RANMAR_MASK;
    g->L[g->head] = v;
    g->head = (g->head + 1) % 97;
    g->C = g->C >= ORC_RANMAR_CD ? g->C - ORC_RANMAR_CD : g->C + ORC_RANMAR_CM - ORC_RANMAR_CD;
    return (v - g->C) & ORC_RANMAR_MASK;
}

static void ranmar_cursor_window(const ranmar_cursor *g, uint32_t window[97])
{
    for (int i = 0; i < 97; i++)
        window[i] = g->L[(g->head + (unsigned)i) % 97];
}

void orc_ranmar_step_to(const uint32_t window0[97], uint64_t n,
                        uint32_t window[97], uint32_t *C)
{
    ranmar_cursor g;
    ranmar_cursor_set(&g, window0, ORC_RANMAR_C0);
    for (uint64_t t = 0; t < n; t++)
        (void)ranmar_next(&g);
    ranmar_cursor_window(&g, window);
    *C = g.C;
}

/* r <- r * q mod (x^97 + x^64 - 1), coefficients mod 2^24: the product of
 * degree <= 192, then every term x^d with d >= 97 folded down by
 * x^d = x^(d-97) - x^(d-33), from the top. */
static void ranmar_polymulmod(uint32_t r[97], const uint32_t q[97])
{
    uint32_t prod[193];
    memset(prod, 0, sizeof prod);
    for (int i = 0; i < 97; i++)
        for (int j = 0; j < 97; j++)
            prod[i + j] += r[i] * q[j];
    for (int d = 192; d >= 97; d--) {
        prod[d - 97] += prod[d];
        prod[d - 33] -= prod[d];
    }
    for (int i = 0; i < 97; i++)
        r[i] = prod[i] & ORC_RANMAR_MASK;
}

void orc_ranmar_jump(const uint32_t window0[97], uint64_t n_lo, uint64_t n_hi,
                     uint32_t window[97], uint32_t *C)
{
    /* r = x^n mod P by square-and-multiply over the bits of n */
    uint32_t r[97], x[97];
    memset(r, 0, sizeof r);
    memset(x, 0, sizeof x);
    r[0] = 1;
    x[1] = 1;
    for (int bit = 127; bit >= 0; bit--) {
        uint32_t sq[97];
        memcpy(sq, r, sizeof sq);
        ranmar_polymulmod(r, sq);
        uint64_t word = bit >= 64 ? n_hi : n_lo;
        if ((word >> (bit & 63)) & 1u)
            ranmar_polymulmod(r, x);
    }
    /* window[s] = L[n - 96 + s] = sum_i (x^(n+s) mod P)_i L[-96 + i] */
    for (int s = 0; s < 97; s++) {
        uint32_t acc = 0;
        for (int i = 0; i < 97; i++)
            acc += r[i] * window0[i];
        window[s] = acc & ORC_RANMAR_MASK;
        ranmar_polymulmod(r, x);
    }
    *C = ranmar_c_at(n_lo, n_hi);
}

void orc_ranmar_words(const uint32_t window0[97], uint64_t first,
                      uint64_t count, uint32_t *out)
{
    uint32_t window[97], C;
    orc_ranmar_jump(window0, first, 0, window, &C);
    ranmar_cursor g;
    ranmar_cursor_set(&g, window, C);
    for (uint64_t t = 0; t < count; t++)
        out[t] = ranmar_next(&g);
}

/* ======================================================================
 * PRNGD.
 * ====================================================================== */

/* Exact round-to-nearest-even of (2^2w - 1) / (D * 2^2w): the factor
 * (1 - k') / [trunc((a - a0 - 2k)/k) + b - b0] of Eq. (5), with k' = k^2,
 * in integer units.  The paper computes this part of Z at compile time;
 * here it is computed once per stream, exactly. */
double orc_scale(int w, uint64_t D)
{
    u128 num = ((u128)1 << (2 * w)) - 1;
    /* choose s so that q = floor(num * 2^s / D) has exactly 53 bits */
    for (int s = 52; s >= -64; s--) {
        u128 n2 = s >= 0 ? num << s : num;
        u128 d2 = s >= 0 ? (u128)D : (u128)D << (-s);
        u128 q = n2 / d2, r = n2 % d2;
        if (q >= ((u128)1 << 53))
            continue;                  /* too many bits: smaller s */
        if (q < ((u128)1 << 52))
            return 0.0;                /* cannot happen for num > D */
        if (2 * r > d2 || (2 * r == d2 && (q & 1u)))
            q += 1;                    /* round half to even */
        return ldexp((double)(uint64_t)q, -s - 2 * w);
    }
    return 0.0;
}

/* Exact RN(1 / D) for D >= 2: q = floor(2^s / D) with exactly 53 bits,
 * rounded half to even, times 2^-s. */
double orc_recip(uint64_t D)
{
    if (D < 2)
        return D == 1 ? 1.0 : 0.0;
    for (int s = 126; s >= 53; s--) {
        u128 n2 = (u128)1 << s;
        u128 q = n2 / D, r = n2 % D;
        if (q >= ((u128)1 << 53))
            continue;
        if (q < ((u128)1 << 52))
            return 0.0;                /* cannot happen: s decreases by one */
        if (2 * r > (u128)D || (2 * r == (u128)D && (q & 1u)))
            q += 1;
        return ldexp((double)(uint64_t)q, -s);
    }
    return 0.0;
}

int orc_set_consume(orc_stream *s, int consume)
{
    if (consume != ORC_CONSUME_PAIR && consume != ORC_CONSUME_SINGLE)
        return -1;
    if (consume == ORC_CONSUME_SINGLE && s->generator != ORC_GEN_PHILOX &&
        s->generator != ORC_GEN_MRG32K3A && s->generator != ORC_GEN_ENUMERATE)
        return -1;
    if (consume == ORC_CONSUME_SINGLE && s->arity == 3)
        return -1;
    s->consume = consume;
    return 0;
}

uint64_t orc_word(const orc_stream *s, uint64_t j)
{
    uint64_t x1, x2;
    uint32_t st[6], o;
    switch (s->generator) {
    case ORC_GEN_PHILOX:
        return philox_word(s->seed, s->stream, j) >> (32 - s->w);
    case ORC_GEN_MRG32K3A:
        memcpy(st, s->mrg, sizeof st);
        {
            uint64_t e[1] = { j };
            orc_mrg_jump(st, e, 1);
        }
        orc_mrg_outputs(st, 1, &o);
        return o;
    case ORC_GEN_RANMAR:
        orc_ranmar_words(s->ranmar, j, 1, &o);
        return o;
    default:
        if (s->arity == 3) {
            /* triple t = j / 3 is (t >> 2w, t >> w, t) mod 2^w */
            uint64_t t = j / 3, mask = (1ull << s->w) - 1;
            return (t >> (s->w * (2 - (int)(j % 3)))) & mask;
        }
        orc_pair(s, j / 2, &x1, &x2);
        return j % 2 ? x2 : x1;
    }
}

/* Algorithm 1 word by word: draw r1 until it is accepted, then r2 is the
 * next word.  The counter is the next word index. */
static void fill_single(orc_stream *s, uint64_t n, double *out, uint64_t *accepted_index)
{
    uint64_t c = s->counter, made = 0;
    uint32_t st[6];
    int mrg = s->generator == ORC_GEN_MRG32K3A;
    if (mrg) {
        memcpy(st, s->mrg, sizeof st);
        uint64_t e[1] = { c };
        orc_mrg_jump(st, e, 1);
    }
    while (made < n) {
        uint64_t r1, r2;
        uint32_t o;
        if (mrg) {
            orc_mrg_outputs(st, 1, &o);
            r1 = o;
        } else {
            r1 = orc_word(s, c);
        }
        c++;
        if (!orc_accept(s, r1))
            continue;
        if (mrg) {
            orc_mrg_outputs(st, 1, &o);
            r2 = o;
        } else {
            r2 = orc_word(s, c);
        }
        c++;
        out[made] = orc_map(s, r1, r2);
        if (accepted_index)
            accepted_index[made] = c - 2;
        made++;
    }
    s->counter = c;
}

int orc_set_map(orc_stream *s, int map)
{
    if (map != ORC_MAP_EQ5 && map != ORC_MAP_EQ4 && map != ORC_MAP_ONE_MINUS)
        return -1;
    if (s->arity == 3 && map != ORC_MAP_EQ5)
        return -1;
    s->map = map;
    return 0;
}

static int finish_init(orc_stream *s)
{
    if (s->w < 1 || s->w > 32 || s->a < s->a0 || s->b < s->b0)
        return -1;
    uint64_t two_w = 1ull << s->w;
    /* the accepted region must be non-empty; x2 must vary (Eq. (5) maps
     * x1 = a0 + k, not a0, to zero, which needs x1 = a0 rejected) and its
     * range must stay below one x1 step (the rejection intervals of
     * Section 2 assume k(b - b0) < 1) */
    if (s->a - s->a0 < 2 || s->a - s->a0 >= two_w || s->b == s->b0 ||
        s->b - s->b0 >= two_w)
        return -1;
    s->D = (s->a - s->a0 - 2) * two_w + (s->b - s->b0);
    s->S = orc_scale(s->w, s->D);
    /* Eq. (4) multiplied through by 2^w: z' = (x1 2^w + x2 - a0 2^w - b) /
     * ((a - a0) 2^w - (b - b0)), with the division folded into RN(1/D4) */
    s->D4 = (s->a - s->a0) * two_w - (s->b - s->b0);
    s->S4 = orc_recip(s->D4);
    s->map = ORC_MAP_EQ5;
    s->consume = ORC_CONSUME_PAIR;
    s->arity = 2;
    return 0;
}

int orc_init_ranges(orc_stream *s, int w, uint64_t a0, uint64_t a,
                    uint64_t b0, uint64_t b)
{
    memset(s, 0, sizeof *s);
    s->generator = -1;
    s->w = w;
    s->a0 = a0; s->a = a; s->b0 = b0; s->b = b;
    return finish_init(s);
}

/* Ranges are the extreme values each base generator can produce, which is
 * what the paper's min and max are (Algorithm 1 parameters). */
int orc_init(orc_stream *s, int generator, int w, uint64_t seed,
             uint32_t stream, uint64_t counter)
{
    memset(s, 0, sizeof *s);
    s->generator = generator;
    s->w = w;
    s->seed = seed;
    s->stream = stream;
    s->counter = counter;
    if (w < 2 || w > 32)
        return -1;
    uint64_t top = (1ull << w) - 1;
    switch (generator) {
    case ORC_GEN_PHILOX:
        s->a0 = 0; s->a = top; s->b0 = 0; s->b = top;
        break;
    case ORC_GEN_MRG32K3A:
        if (w != 32) return -1;
        s->a0 = 1; s->a = ORC_M1; s->b0 = 1; s->b = ORC_M1;
        break;
    case ORC_GEN_MIXED:
        if (w != 32) return -1;
        s->a0 = 0; s->a = top; s->b0 = 1; s->b = ORC_M1;
        break;
    case ORC_GEN_ENUMERATE:
        if (w > 16) return -1;
        s->a0 = 0; s->a = top; s->b0 = 0; s->b = top;
        break;
    case ORC_GEN_RANMAR:
        if (w != 24) return -1;
        s->a0 = 0; s->a = top; s->b0 = 0; s->b = top;
        {
            uint32_t ij, kl;
            orc_ranmar_stream_seeds(seed, stream, &ij, &kl);
            orc_ranmar_seed(ij, kl, s->ranmar);
        }
        break;
    default:
        return -1;
    }
    if (generator == ORC_GEN_MRG32K3A || generator == ORC_GEN_MIXED)
        orc_mrg_stream_base(seed, stream, s->mrg);
    return finish_init(s);
}

/* MRG outputs per pair: both words for the MRG-only generator, x2 only for
 * the mixed one. */
static uint64_t mrg_per_pair(const orc_stream *s)
{
    return s->generator == ORC_GEN_MRG32K3A ? 2 : 1;
}

static void mrg_state_at(const orc_stream *s, uint64_t position,
                         uint32_t st[6])
{
    memcpy(st, s->mrg, sizeof s->mrg);
    uint64_t e[1] = { position };
    orc_mrg_jump(st, e, 1);
}

/* Pair p of the stream (random access; slow for the MRG generators). */
void orc_pair(const orc_stream *s, uint64_t p, uint64_t *x1, uint64_t *x2)
{
    int shift = 32 - s->w;
    uint32_t st[6], o[2];
    switch (s->generator) {
    case ORC_GEN_PHILOX:   /* words 2p and 2p + 1, i.e. block p / 2 */
        *x1 = philox_lane(s->seed, s->stream, p / 2, 2 * (unsigned)(p % 2)) >> shift;
        *x2 = philox_lane(s->seed, s->stream, p / 2, 2 * (unsigned)(p % 2) + 1) >> shift;
        break;
    case ORC_GEN_MRG32K3A:
        /* output 2p is produced by the step from position 2p to 2p + 1 */
        mrg_state_at(s, 2 * p, st);
        orc_mrg_outputs(st, 2, o);
        *x1 = o[0];
        *x2 = o[1];
        break;
    case ORC_GEN_MIXED:
        *x1 = philox_word(s->seed, s->stream, p);
        mrg_state_at(s, p, st);
        orc_mrg_outputs(st, 1, o);
        *x2 = o[0];
        break;
    case ORC_GEN_ENUMERATE:
        *x1 = (p >> s->w) & ((1ull << s->w) - 1);
        *x2 = p & ((1ull << s->w) - 1);
        break;
    case ORC_GEN_RANMAR: {
        uint32_t wd[2];
        {
            u128 first = (u128)2 * p;
            uint32_t window[97], C;
            orc_ranmar_jump(s->ranmar, (uint64_t)first, (uint64_t)(first >> 64), window, &C);
            ranmar_cursor g;
            ranmar_cursor_set(&g, window, C);
            wd[0] = ranmar_next(&g);
            wd[1] = ranmar_next(&g);
        }
        *x1 = wd[0];
        *x2 = wd[1];
        break;
    }
    default:
        *x1 = *x2 = 0;
    }
}

/* Section 2: pairs whose x1 lies in x1 < a0 + k(b - b0) or
 * x1 > a - k(b - b0) are rejected.  Multiplied through by 2^w the test is
 * exact in integers.  For discrete x1 with 0 < b - b0 < 2^w it reduces to
 * rejecting x1 = a0 and x1 = a, the paper's practical rule. */
int orc_accept(const orc_stream *s, uint64_t x1)
{
    i128 scaled = (i128)x1 << s->w;
    i128 width = (i128)(s->b - s->b0);
    i128 lo = ((i128)s->a0 << s->w) + width;
    i128 hi = ((i128)s->a << s->w) - width;
    return !(scaled < lo || scaled > hi);
}

/* Eq. (5) in integer units: the numerator trunc[(x1 - a0 - k)/k] + x2 - b0
 * is the exact integer N = (x1 - a0 - 1) 2^w + (x2 - b0); the output is
 * RN(RN(N) * S) with S the folded constant, forced below 1 when rounding
 * reaches 1.0 (possible only for w > 26, where 1 - k^2 is not a double). */
double orc_map(const orc_stream *s, uint64_t x1, uint64_t x2)
{
    if (s->map == ORC_MAP_EQ4) {
        /* numerator of Eq. (4) in integer units; positive for accepted x1 */
        uint64_t N4 = ((x1 - s->a0) << s->w) + x2 - s->b;
        double z = (double)N4 * s->S4;
        if (z >= 1.0)
            z = 0x1.fffffffffffffp-1;
        return z;
    }
    uint64_t N = ((x1 - s->a0 - 1) << s->w) + (x2 - s->b0);
    double z = (double)N * s->S;
    if (z >= 1.0)
        z = 0x1.fffffffffffffp-1;
    if (s->map == ORC_MAP_ONE_MINUS)
        z = 1.0 - z;
    return z;
}

/* Algorithm 1 with pair consumption: draw the next pair, drop it if x1 is
 * in a rejection interval (both of its words are used up), otherwise map
 * it.  The walk stops once n outputs exist or, when `bounded`, once pair
 * `pair_end` is reached (that pair is not examined); returns the outputs
 * made and leaves s->counter at the first pair not examined. */
static uint64_t fill_pairs(orc_stream *s, uint64_t n, int bounded, uint64_t pair_end,
                           double *out, uint64_t *accepted_index)
{
    int mrg = s->generator == ORC_GEN_MRG32K3A || s->generator == ORC_GEN_MIXED;
    uint32_t st[6];
    int shift = 32 - s->w;
    ranmar_cursor rm;
    if (s->generator == ORC_GEN_RANMAR) {
        /* words 2 counter, 2 counter + 1, ... from the window there */
        u128 first = (u128)2 * s->counter;
        uint32_t window[97], C;
        orc_ranmar_jump(s->ranmar, (uint64_t)first, (uint64_t)(first >> 64), window, &C);
        ranmar_cursor_set(&rm, window, C);
    }
    if (mrg) {
        /* position r * counter may need 65 bits */
        u128 pos = (u128)mrg_per_pair(s) * s->counter;
        uint64_t e[2] = { (uint64_t)pos, (uint64_t)(pos >> 64) };
        memcpy(st, s->mrg, sizeof st);
        orc_mrg_jump(st, e, 2);
    }
    uint64_t made = 0, p = s->counter;
    while (made < n && !(bounded && p >= pair_end)) {
        uint64_t x1, x2;
        uint32_t o[2];
        switch (s->generator) {
        case ORC_GEN_PHILOX:
            x1 = philox_lane(s->seed, s->stream, p / 2, 2 * (unsigned)(p % 2)) >> shift;
            x2 = philox_lane(s->seed, s->stream, p / 2, 2 * (unsigned)(p % 2) + 1) >> shift;
            break;
        case ORC_GEN_MRG32K3A:
            orc_mrg_outputs(st, 2, o);
            x1 = o[0];
            x2 = o[1];
            break;
        case ORC_GEN_MIXED:
            x1 = philox_word(s->seed, s->stream, p);
            orc_mrg_outputs(st, 1, o);
            x2 = o[0];
            break;
        case ORC_GEN_RANMAR:
            x1 = ranmar_next(&rm);
            x2 = ranmar_next(&rm);
            break;
        default:
            orc_pair(s, p, &x1, &x2);
            break;
        }
        p++;
        if (!orc_accept(s, x1))
            continue;
        out[made] = orc_map(s, x1, x2);
        if (accepted_index)
            accepted_index[made] = p - 1;
        made++;
    }
    s->counter = p;
    return made;
}

/* ======================================================================
 * Three words per output: the two-word method applied twice (see the
 * header for the reading).
 * ====================================================================== */

/* Round-to-nearest-even of a 128-bit integer: keep its 53 leading bits,
 * look at the rest. */
double orc_rn_u128(uint64_t hi, uint64_t lo)
{
    u128 v = ((u128)hi << 64) | lo;
    int bits = 0;
    for (u128 t = v; t; t >>= 1)
        bits++;
    if (bits <= 53)
        return (double)(uint64_t)v;            /* exact */
    int sh = bits - 53;
    u128 q = v >> sh;
    u128 rem = v - (q << sh);
    u128 half = (u128)1 << (sh - 1);
    if (rem > half || (rem == half && (q & 1u)))
        q += 1;                                /* may reach 2^53: still exact */
    return ldexp((double)(uint64_t)q, sh);
}

/* RN((2^3w - 1) / (D 2^3w)) by binary long division of num = 2^3w - 1 by
 * D: the quotient is normalised to [1, 2), its 52 fraction bits are found
 * one by one, and the remainder decides the rounding (half to even). */
double orc_scale3(int w, uint64_t D_hi, uint64_t D_lo)
{
    u128 D = ((u128)D_hi << 64) | D_lo;
    u128 num = ((u128)1 << (3 * w)) - 1;
    if (D == 0 || D > num)
        return 0.0;
    int e = 0;                                 /* num / (D 2^e) in [1, 2) */
    while ((D << (e + 1)) <= num)
        e++;
    u128 d = D << e;
    u128 q = 1, r = num - d;
    for (int i = 0; i < 52; i++) {
        r <<= 1;
        q <<= 1;
        if (r >= d) {
            q |= 1;
            r -= d;
        }
    }
    if (2 * r > d || (2 * r == d && (q & 1u)))
        q += 1;
    return ldexp((double)(uint64_t)q, e - 52 - 3 * w);
}

/* Section 2's rejection intervals, exact in integers: the inner pair
 * (x2, x3) with x3's span a - a0 (scaled by 2^w); the outer pair (x1, y)
 * with y's span Y1 - Y0 (scaled by 2^2w). */
int orc_accept3(const orc_stream *s, uint64_t x1, uint64_t x2)
{
    int w = s->w;
    i128 span = (i128)(s->a - s->a0);
    i128 x2s = (i128)x2 << w;
    if (x2s < ((i128)s->a0 << w) + span || x2s > ((i128)s->a << w) - span)
        return 0;
    i128 yspan = ((i128)(s->a - s->a0 - 2) << w) + span;       /* Y1 - Y0 */
    i128 x1s = (i128)x1 << (2 * w);
    if (x1s < ((i128)s->a0 << (2 * w)) + yspan || x1s > ((i128)s->a << (2 * w)) - yspan)
        return 0;
    return 1;
}

double orc_map3(const orc_stream *s, uint64_t x1, uint64_t x2, uint64_t x3)
{
    int w = s->w;
    u128 Y = ((u128)x2 << w) + x3;
    u128 Y0 = ((u128)(s->a0 + 1) << w) + s->a0;
    u128 N = ((u128)(x1 - s->a0 - 1) << (2 * w)) + (Y - Y0);
    double z = orc_rn_u128((uint64_t)(N >> 64), (uint64_t)N) * s->S3;
    if (z >= 1.0)
        z = 0x1.fffffffffffffp-1;
    return z;
}

int orc_set_arity(orc_stream *s, int arity)
{
    if (arity == 2) {
        s->arity = 2;
        return 0;
    }
    if (arity != 3 || s->consume != ORC_CONSUME_PAIR || s->map != ORC_MAP_EQ5 ||
        (s->generator != ORC_GEN_PHILOX && s->generator != ORC_GEN_MRG32K3A &&
         s->generator != ORC_GEN_ENUMERATE))
        return -1;
    int w = s->w;
    u128 yspan = ((u128)(s->a - s->a0 - 2) << w) + (s->a - s->a0);
    u128 D = ((u128)(s->a - s->a0 - 2) << (2 * w)) + yspan;
    s->D3_hi = (uint64_t)(D >> 64);
    s->D3_lo = (uint64_t)D;
    s->S3 = orc_scale3(w, s->D3_hi, s->D3_lo);
    s->arity = 3;
    return 0;
}

/* The next n outputs of a three-word stream, triple by triple (at most n,
 * and only triples below `end` when bounded); returns how many. */
static uint64_t fill_triples(orc_stream *s, uint64_t n, int bounded, uint64_t end,
                             double *out, uint64_t *accepted_index)
{
    int mrg = s->generator == ORC_GEN_MRG32K3A;
    uint32_t st[6];
    if (mrg) {
        u128 pos = (u128)3 * s->counter;
        uint64_t e[2] = { (uint64_t)pos, (uint64_t)(pos >> 64) };
        memcpy(st, s->mrg, sizeof st);
        orc_mrg_jump(st, e, 2);
    }
    uint64_t made = 0, t = s->counter;
    while (made < n && !(bounded && t >= end)) {
        uint64_t x[3];
        for (int i = 0; i < 3; i++) {
            if (mrg) {
                uint32_t o;
                orc_mrg_outputs(st, 1, &o);
                x[i] = o;
            } else {
                x[i] = orc_word(s, 3 * t + (uint64_t)i);
            }
        }
        t++;
        if (!orc_accept3(s, x[0], x[1]))
            continue;
        out[made] = orc_map3(s, x[0], x[1], x[2]);
        if (accepted_index)
            accepted_index[made] = t - 1;
        made++;
    }
    s->counter = t;
    return made;
}

void orc_fill(orc_stream *s, uint64_t n, double *out,
              uint64_t *accepted_index)
{
    if (s->arity == 3) {
        fill_triples(s, n, 0, 0, out, accepted_index);
        return;
    }
    if (s->consume == ORC_CONSUME_SINGLE) {
        fill_single(s, n, out, accepted_index);
        return;
    }
    fill_pairs(s, n, 0, 0, out, accepted_index);
}

uint64_t orc_fill_pairs(orc_stream *s, uint64_t pair_end, uint64_t max_out, double *out)
{
    if (s->consume == ORC_CONSUME_SINGLE)
        return 0;
    if (s->arity == 3)
        return fill_triples(s, max_out, 1, pair_end, out, NULL);
    return fill_pairs(s, max_out, 1, pair_end, out, NULL);
}
