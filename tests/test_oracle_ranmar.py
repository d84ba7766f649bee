"""The oracle's RANMAR base generator and PRNGD on its words.

RANMAR (Marsaglia, Zaman and Tsang 1990, in the form F. James gives in his
1990 review) is one of the 24-bit generators the paper names as suitable
base generators (Section 2).  Pins:

* the generator's own published check values (seeds 1802 and 9373: the six
  numbers after the first 20000), a fixture under ``golden/``;
* the window at any word position by the jump polynomial equals the window
  reached by stepping, at positions around the lags (0, 1, 32, 33, 96, 97,
  98, 193, 194) and at random ones;
* the arithmetic part C[n] has the closed form (C[0] - 7654321 n) mod
  16777213, checked against stepping at large n through the jump;
* the seeding convention of a PRNGD stream (seed, stream) reaches the
  published sequence;
* PRNGD on RANMAR words: pair p is words (2p, 2p + 1), x1 in {0, 2^24 - 1}
  is rejected and consumes the pair, Eq. (5) maps the rest -- checked
  against a brute-force walk over the words with exact rationals.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
MASK = (1 << 24) - 1


def golden():
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "ranmar_check_values.txt"))
            if ln.strip() and not ln.startswith("#")]
    ij, kl, skip = (int(x) for x in rows[0])
    return ij, kl, skip, [int(r[0]) for r in rows[1:]]


def test_published_check_values():
    ij, kl, skip, values = golden()
    w0 = O.ranmar_seed(ij, kl)
    assert list(O.ranmar_words(w0, skip, len(values))) == values


def test_seed_values_are_24_bit_and_differ_by_seed():
    a, b = O.ranmar_seed(1802, 9373), O.ranmar_seed(1802, 9374)
    assert a.max() < 2**24 and b.max() < 2**24
    assert not np.array_equal(a, b)


def python_step(window, C, n):
    """Plain Python stepping from (window, C), n words: returns the words."""
    L = [int(x) for x in window]
    out = []
    for _ in range(n):
        v = (L[0] - L[64]) & MASK
        L = L[1:] + [v]
        C = C - 7654321 if C >= 7654321 else C - 7654321 + 16777213
        out.append((v - C) & MASK)
    return out, L, C


def test_stepping_matches_a_plain_python_walk():
    w0 = O.ranmar_seed(1802, 9373)
    words, L, C = python_step(w0, 362436, 500)
    assert list(O.ranmar_words(w0, 0, 500)) == words
    win, c = O.ranmar_step_to(w0, 500)
    assert list(win) == L and c == C


@pytest.mark.parametrize("n", [0, 1, 2, 32, 33, 34, 64, 96, 97, 98, 193, 194, 1000, 4097])
def test_jump_equals_stepping_around_the_lags(n):
    w0 = O.ranmar_seed(17, 4242)
    a, ca = O.ranmar_step_to(w0, n)
    b, cb = O.ranmar_jump(w0, n)
    assert np.array_equal(a, b) and ca == cb


def test_jump_equals_stepping_at_random_positions():
    rnd = np.random.default_rng(5)
    for _ in range(6):
        ij, kl = int(rnd.integers(0, 31329)), int(rnd.integers(0, 30082))
        n = int(rnd.integers(0, 300000))
        w0 = O.ranmar_seed(ij, kl)
        a, ca = O.ranmar_step_to(w0, n)
        b, cb = O.ranmar_jump(w0, n)
        assert np.array_equal(a, b) and ca == cb, (ij, kl, n)


def test_jumps_compose():
    # the window at m + n reached from the window at m by stepping n more
    w0 = O.ranmar_seed(3, 5)
    m = 2**40 + 12345
    wm, cm = O.ranmar_jump(w0, m)
    words, L, C = python_step(wm, cm, 300)
    w1, c1 = O.ranmar_jump(w0, m + 300)
    assert list(w1) == L and c1 == C
    assert list(O.ranmar_words(w0, m, 300)) == words


def test_arithmetic_part_closed_form():
    w0 = O.ranmar_seed(0, 0)
    for n in [0, 1, 2, 3, 1000, 2**33 + 1, 2**64 + 7]:
        _, c = O.ranmar_jump(w0, n)
        assert c == (362436 - 7654321 * n) % 16777213


def test_stream_seeding_reaches_the_published_sequence():
    ij, kl, skip, values = golden()
    s = ij * 30082 + kl
    assert O.ranmar_stream_seeds(0, s) == (ij, kl)
    assert O.ranmar_stream_seeds(1, s) == divmod((2**32 + s) % (31329 * 30082), 30082)
    st = O.PRNGD(O.GEN_RANMAR, 24, seed=0, stream=s)
    assert [st.word(skip + i) for i in range(len(values))] == values


def eq5(x1, x2):
    """Eq. (5) at w = 24 with a0 = b0 = 0, a = b = 2^24 - 1, exact then
    rounded once: N = (x1 - 1) 2^24 + x2, D = (2^24 - 3) 2^24 + 2^24 - 1."""
    N = (x1 - 1) * 2**24 + x2
    D = (2**24 - 3) * 2**24 + (2**24 - 1)
    S = float(Fraction(2**48 - 1, D * 2**48))
    return float(N) * S


@pytest.mark.parametrize("seed,stream,counter", [(0, 0, 0), (7, 3, 5), (2**40 + 1, 77, 10**6 + 1)])
def test_prngd_on_ranmar_words(seed, stream, counter):
    st = O.PRNGD(O.GEN_RANMAR, 24, seed=seed, stream=stream, counter=counter)
    assert st.ranges == (0, MASK, 0, MASK)
    n = 3000
    out = st.fill(n)
    ij, kl = O.ranmar_stream_seeds(seed, stream)
    words = O.ranmar_words(O.ranmar_seed(ij, kl), 2 * counter, 2 * n + 64)
    expect, p = [], counter
    while len(expect) < n:
        x1, x2 = int(words[2 * (p - counter)]), int(words[2 * (p - counter) + 1])
        p += 1
        if x1 in (0, MASK):
            continue
        expect.append(eq5(x1, x2))
    assert np.array_equal(out, np.array(expect))
    assert st.counter == p


def test_rejected_pairs_consume_both_words():
    # find a rejection (x1 = 0 or 2^24 - 1 occurs once in 2^23 pairs)
    w0 = O.ranmar_seed(*O.ranmar_stream_seeds(0, 0))
    st = O.PRNGD(O.GEN_RANMAR, 24, seed=0, stream=0)
    chunk = 1 << 22
    for base in range(0, 1 << 26, chunk):
        words = O.ranmar_words(w0, 2 * base, 2 * chunk)
        x1 = words[0::2]
        hit = np.flatnonzero((x1 == 0) | (x1 == MASK))
        if hit.size:
            p = base + int(hit[0])
            break
    else:
        pytest.skip("no rejection in the first 2^26 pairs")
    st.counter = p - 2
    out = st.fill(3)
    ws = O.ranmar_words(w0, 2 * (p - 2), 8)
    assert np.array_equal(out, [eq5(int(ws[0]), int(ws[1])), eq5(int(ws[2]), int(ws[3])),
                                eq5(int(ws[6]), int(ws[7]))])
    assert st.counter == p + 2


def test_one_word_consumption_and_three_words_are_refused():
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_RANMAR, 24, consume=O.CONSUME_SINGLE)
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_RANMAR, 24, arity=3)
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_RANMAR, 32)
