// prngd_ranmar_host.cpp -- host side of the RANMAR base generator: the seed
// window of a sequence, the window at any word position (the jump
// polynomial), and the rows of the jump table the fill kernels read.
//
// RANMAR: Marsaglia, Zaman, Tsang, Stat. Prob. Lett. 9 (1990) 35, in the
// form of F. James, Comput. Phys. Commun. 60 (1990) 329.  In integer units
// of 2^-24: L[n] = (L[n-97] - L[n-33]) mod 2^24, C[n] = (C[n-1] - 7654321)
// mod 16777213 with C[0] = 362436, word j = (L[j+1] - C[j+1]) mod 2^24.
// The recurrence of L is the shift relation x^97 = 1 - x^64, so the window
// n words on is given by x^n mod (x^97 + x^64 - 1): L[n - 96 + s] =
// sum_i (x^(n+s) mod P)_i L[-96 + i].
#include <cstdint>
#include <cstring>

#include "prngd_internal.hpp"

namespace prngd {

namespace {

constexpr uint32_t kSeqIJ = 31329;   // seeds ij in [0, 31328]
constexpr uint32_t kSeqKL = 30082;   // seeds kl in [0, 30081]

using u128 = unsigned __int128;

// The 97 seed values of sequence (ij, kl): a three-lag Fibonacci generator
// mod 179 and a congruential generator mod 169 give one bit per step (set
// when (l m) mod 64 >= 32), 24 bits per value, the first bit the highest;
// the values in turn are L[0], L[-1], ..., L[-96].
void seed_window(uint32_t ij, uint32_t kl, uint32_t win[97])
{
    uint32_t i = (ij / 177) % 177 + 2, j = ij % 177 + 2;
    uint32_t k = (kl / 169) % 178 + 1, l = kl % 169;
    for (int v = 0; v < 97; ++v) {
        uint32_t bits = 0;
        for (int b = 0; b < 24; ++b) {
            const uint32_t m = (((i * j) % 179) * k) % 179;
            i = j;
            j = k;
            k = m;
            l = (53 * l + 1) % 169;
            bits = (bits << 1) | ((l * m) % 64 >= 32 ? 1u : 0u);
        }
        win[96 - v] = bits;
    }
}

// A polynomial of degree < 97 over the integers mod 2^24 (mod 2^32 in the
// arithmetic; only the low 24 bits are kept).
struct Poly {
    uint32_t c[97];
};

Poly poly_one()
{
    Poly p{};
    p.c[0] = 1;
    return p;
}

// x^97 = 1 - x^64: fold the terms of degree 97 .. 192 from the top down.
Poly poly_mulmod(const Poly &a, const Poly &b)
{
    uint32_t prod[193] = {};
    for (int i = 0; i < 97; ++i) {
        if (!a.c[i])
            continue;
        for (int j = 0; j < 97; ++j)
            prod[i + j] += a.c[i] * b.c[j];
    }
    for (int d = 192; d >= 97; --d) {
        prod[d - 97] += prod[d];
        prod[d - 33] -= prod[d];
    }
    Poly r;
    for (int i = 0; i < 97; ++i)
        r.c[i] = prod[i] & kRanmarMask;
    return r;
}

// x * a mod P: a shift, and the top coefficient folded.
Poly poly_times_x(const Poly &a)
{
    Poly r;
    const uint32_t top = a.c[96];
    r.c[0] = top;
    for (int i = 1; i < 97; ++i)
        r.c[i] = a.c[i - 1];
    r.c[64] = (r.c[64] - top) & kRanmarMask;
    return r;
}

Poly poly_x_pow(u128 n)
{
    Poly r = poly_one();
    int top = 127;
    while (top >= 0 && !((n >> top) & 1u))
        --top;
    for (int b = top; b >= 0; --b) {
        r = poly_mulmod(r, r);
        if ((n >> b) & 1u)
            r = poly_times_x(r);
    }
    return r;
}

uint32_t c_at(u128 n)
{
    const uint64_t t = uint64_t(n % kRanmarCM) * kRanmarCD % kRanmarCM;
    return uint32_t((uint64_t(kRanmarC0) + kRanmarCM - t) % kRanmarCM);
}

}  // namespace

void ranmar_sequence_of(uint64_t seed, uint32_t stream, uint32_t *ij, uint32_t *kl)
{
    const u128 s = ((u128(seed) << 32) | stream) % (u128(kSeqIJ) * kSeqKL);
    *ij = uint32_t(s / kSeqKL);
    *kl = uint32_t(s % kSeqKL);
}

void ranmar_window_at(uint64_t seed, uint32_t stream, uint64_t word_lo, uint64_t word_hi,
                      uint32_t out[kRanmarRow])
{
    uint32_t ij = 0, kl = 0, w0[97];
    ranmar_sequence_of(seed, stream, &ij, &kl);
    seed_window(ij, kl, w0);
    const u128 n = (u128(word_hi) << 64) | word_lo;
    std::memset(out, 0, kRanmarRow * sizeof(uint32_t));
    if (n == 0) {
        std::memcpy(out, w0, sizeof w0);
    } else {
        Poly r = poly_x_pow(n);
        for (int s = 0; s < 97; ++s) {
            uint32_t acc = 0;
            for (int i = 0; i < 97; ++i)
                acc += r.c[i] * w0[i];
            out[s] = acc & kRanmarMask;
            r = poly_times_x(r);
        }
    }
    out[97] = c_at(n);
}

void ranmar_jump_rows(uint32_t seg_pairs, uint32_t first, uint32_t count, uint32_t *rows)
{
    const u128 step = u128(2) * seg_pairs;
    const Poly x_step = poly_x_pow(step);
    Poly r = poly_x_pow(step * first);
    for (uint32_t g = first; g < first + count; ++g) {
        uint32_t *row = rows + size_t(g - first) * kRanmarRow;
        std::memset(row, 0, kRanmarRow * sizeof(uint32_t));
        std::memcpy(row, r.c, sizeof r.c);
        row[97] = uint32_t(uint64_t(step * g % kRanmarCM) * kRanmarCD % kRanmarCM);
        r = poly_mulmod(r, x_step);
    }
}

}  // namespace prngd
