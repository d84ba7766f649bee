"""Pins of the oracle's three-words-per-output form (the paper's Conclusion:
more than two PRNs combined), the two-word method applied twice.

Reading (also in the oracle header): the inner pair (x2, x3) is accepted by
Section 2's rule into y = x2 + k x3, a PRN of resolution k^2; the outer pair
(x1, y) is accepted by the same rule with y's span, and Eq. (5) maps
z = x1 + k y with the resulting resolution k' = k^3.  In integer units
N3 = (x1 - a0 - 1) 2^2w + (x2 - a0 - 1) 2^w + (x3 - a0),
D3 = (a - a0 - 2) 2^2w + (a - a0 - 2) 2^w + (a - a0), z' = RN(RN(N3) S3),
S3 = RN((1 - 2^-3w) / D3), forced below 1.

What pins it, besides itself:
* its 128-bit rounding equals Python's correctly rounded int -> float;
* S3 equals the correctly rounded exact rational, for the real D3 and for
  random divisors;
* exhaustive enumeration at w = 4 and w = 5: exactly the triples with x1 or
  x2 in {a0, a} are rejected (the closed-form fraction 1 - (1 - 2/2^w)^2),
  the accepted N3 are exactly the grid {i 2^2w + j 2^w + l}, each once, in
  increasing order, and every output lies within the rounding bound of the
  exact N3 (1 - k^3) / D3;
* the end points: N3 = 0 gives +0, N3 = D3 gives 1 - k^3 within an ulp
  (forced below 1 where 1 - k^3 rounds to 1);
* Philox and MRG32k3a streams: every output within the same bound of the
  exact value computed from the generators' own words, and the counter
  counts triples;
* chi-square and Kolmogorov-Smirnov on 2^20 outputs.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

BELOW_ONE = float.fromhex("0x1.fffffffffffffp-1")


def D3_of(w, a0, a):
    return (a - a0 - 2) * 2**(2 * w) + (a - a0 - 2) * 2**w + (a - a0)


def N3_of(w, a0, x1, x2, x3):
    return (x1 - a0 - 1) * 2**(2 * w) + (x2 - a0 - 1) * 2**w + (x3 - a0)


def ulp(x):
    return math.ulp(x) if x != 0 else 2.0**-1074


def within_bound(z, N, D, w):
    """z = RN(RN(N) S3) with S3 = RN((1 - k^3)/D): two roundings of N and
    one of S3 and one of the product -- at most 3/2 ulp from the exact
    value (1 ulp when N is exact, 3 w <= 53)."""
    exact = Fraction(N) * (1 - Fraction(1, 2**(3 * w))) / D
    if exact >= 1:
        return z == BELOW_ONE
    return abs(Fraction(z) - exact) <= Fraction(3, 2) * Fraction(ulp(z))


def test_rn_u128_is_correct_rounding():
    rnd = random.Random(3)
    vals = [0, 1, 2**53 - 1, 2**53, 2**53 + 1, 2**53 + 2, 2**54 + 2, 2**54 + 6,
            2**64 - 1, 2**96 - 1, 2**127 + 2**74 + 2**73, 2**128 - 1]
    for bits in range(1, 129):
        for _ in range(12):
            vals.append(rnd.getrandbits(bits))
    # exact ties at several positions: half-even decides
    for sh in (1, 2, 11, 40, 70):
        for q in (2**52 + 1, 2**52 + 2, 2**53 - 1):
            vals.append((2 * q + 1) << (sh - 1) if sh > 1 else 2 * q + 1)
    for v in vals:
        if v >= 2**128:
            continue
        assert O.rn_u128(v) == float(v), hex(v)


@pytest.mark.parametrize("w", [3, 4, 5, 8, 16, 17, 21, 24, 27, 32])
def test_scale3_is_the_correctly_rounded_constant(w):
    D3 = D3_of(w, 0, 2**w - 1)
    s = O.PRNGD(O.GEN_PHILOX, w, arity=3)
    assert s.D3 == D3
    exact = Fraction(2**(3 * w) - 1, D3 * 2**(3 * w))
    assert s.S3 == float(exact)            # Fraction -> float rounds correctly
    rnd = random.Random(w)
    for _ in range(50):
        D = rnd.randrange(2**(3 * w - 3), 2**(3 * w) - 1)
        assert O.scale3(w, D) == float(Fraction(2**(3 * w) - 1, D * 2**(3 * w)))


@pytest.mark.parametrize("w", [4, 5])
def test_exhaustive_enumeration(w):
    a0, a = 0, 2**w - 1
    s = O.PRNGD(O.GEN_ENUMERATE, w, arity=3)
    D3 = D3_of(w, a0, a)
    total = 2**(3 * w)
    kept = (a - a0 - 1)**2 * (a - a0 + 1)
    # rejection fraction in closed form: 1 - (1 - 2/2^w)^2
    assert Fraction(total - kept, total) == 1 - (1 - Fraction(2, 2**w))**2
    out, idx = s.fill(kept, with_index=True)
    # accepted triples: x1 and x2 not in {a0, a}, in order
    expect_idx = [t for t in range(total)
                  if (t >> (2 * w)) not in (a0, a) and ((t >> w) & a) not in (a0, a)]
    assert list(idx) == expect_idx
    assert s.counter == expect_idx[-1] + 1
    N = [N3_of(w, a0, t >> (2 * w), (t >> w) & a, t & a) for t in expect_idx]
    grid = sorted(i * 2**(2 * w) + j * 2**w + l
                  for i in range(a - a0 - 1) for j in range(a - a0 - 1) for l in range(a - a0 + 1))
    assert N == grid                         # every grid value once, in order
    assert np.all(np.diff(out) > 0)          # strictly increasing
    for z, n in zip(out, N):
        assert within_bound(float(z), n, D3, w)
    assert out[0] == 0.0                     # N3 = 0
    assert N[-1] == D3
    assert abs(Fraction(float(out[-1])) - (1 - Fraction(1, 2**(3 * w)))) <= ulp(float(out[-1]))


def test_rejection_rule_is_section_2_applied_twice():
    # exact integer tests of the inner and the outer interval agree with
    # "x1 and x2 not at the range ends" for every width, and at w = 32 for
    # MRG32k3a's range
    for w in (2, 3, 8, 17, 32):
        s = O.PRNGD(O.GEN_PHILOX, w, arity=3)
        top = 2**w - 1
        for x1 in (0, 1, 2, top - 1, top):
            for x2 in (0, 1, top - 1, top):
                assert s.accept3(x1, x2) == (x1 not in (0, top) and x2 not in (0, top))
    m = O.PRNGD(O.GEN_MRG32K3A, 32, arity=3)
    for x1 in (1, 2, O.M1 - 1, O.M1):
        for x2 in (1, 2, O.M1 - 1, O.M1):
            assert m.accept3(x1, x2) == (x1 not in (1, O.M1) and x2 not in (1, O.M1))


@pytest.mark.parametrize("w", [17, 24, 27, 32])
def test_end_points(w):
    s = O.PRNGD(O.GEN_PHILOX, w, arity=3)
    top = 2**w - 1
    assert s.map3(1, 1, 0) == 0.0
    zmax = s.map3(top - 1, top - 1, top)
    one_minus = 1 - Fraction(1, 2**(3 * w))
    if float(one_minus) == 1.0:
        assert zmax == BELOW_ONE
    else:
        assert abs(Fraction(zmax) - one_minus) <= ulp(zmax)
    assert 0.0 < s.map3(1, 1, 1) < 2.0**-(3 * w - 2)


@pytest.mark.parametrize("w,seed,counter", [(17, 42, 0), (24, 7, 12345), (32, 9, 2**40 + 1),
                                            (5, 3, 0)])
def test_philox_triples_against_their_words(w, seed, counter):
    n = 4000
    s = O.PRNGD(O.GEN_PHILOX, w, seed=seed, stream=3, counter=counter, arity=3)
    out = s.fill(n)
    used = s.counter - counter
    words = O.philox_words(seed, 3, 3 * counter, 3 * used)
    x = [int(v) >> (32 - w) for v in words]
    top = 2**w - 1
    D3 = D3_of(w, 0, top)
    k = 0
    for t in range(used):
        x1, x2, x3 = x[3 * t: 3 * t + 3]
        if x1 in (0, top) or x2 in (0, top):
            continue
        assert within_bound(float(out[k]), N3_of(w, 0, x1, x2, x3), D3, w), (t, k)
        k += 1
    assert k == n                            # the counter stopped after output n - 1
    # with 3 w <= 53, RN(N3) is exact and the output is one rounding of N3 S3
    if 3 * w <= 53:
        k = 0
        for t in range(used):
            x1, x2, x3 = x[3 * t: 3 * t + 3]
            if x1 in (0, top) or x2 in (0, top):
                continue
            assert out[k] == float(N3_of(w, 0, x1, x2, x3)) * s.S3
            k += 1


def test_mrg32k3a_triples_against_their_outputs():
    n = 1500
    s = O.PRNGD(O.GEN_MRG32K3A, 32, seed=11, arity=3)
    out = s.fill(n)
    outs, _ = O.mrg_outputs(O.mrg_stream_base(11, 0), 3 * s.counter)
    x = [int(v) for v in outs]
    D3 = D3_of(32, 1, O.M1)
    k = 0
    for t in range(s.counter):
        x1, x2, x3 = x[3 * t: 3 * t + 3]
        if x1 in (1, O.M1) or x2 in (1, O.M1):
            continue
        assert within_bound(float(out[k]), N3_of(32, 1, x1, x2, x3), D3, 32)
        k += 1
    assert k == n


def test_triples_concatenate_and_count_triples():
    a = O.PRNGD(O.GEN_PHILOX, 8, seed=5, arity=3)
    b = O.PRNGD(O.GEN_PHILOX, 8, seed=5, arity=3)
    whole = a.fill(3000)
    parts = np.concatenate([b.fill(1000), b.fill(1), b.fill(1999)])
    assert np.array_equal(whole.view(np.uint64), parts.view(np.uint64))
    assert a.counter == b.counter
    # at w = 8 about 1.6 % of triples are rejected
    assert 3000 < a.counter < 3000 * 1.03


def test_refusals():
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_MIXED, 32, arity=3)
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_PHILOX, 8, map=O.MAP_EQ4, arity=3)
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_PHILOX, 8, consume=O.CONSUME_SINGLE, arity=3)
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_PHILOX, 8, arity=4)


def test_uniformity():
    scipy_stats = pytest.importorskip("scipy.stats")
    z = O.PRNGD(O.GEN_PHILOX, 17, seed=2024, arity=3).fill(1 << 20)
    assert np.all((0.0 <= z) & (z < 1.0))
    counts = np.bincount(np.minimum((z * 1024).astype(np.int64), 1023), minlength=1024)
    chi2 = float(((counts - len(z) / 1024) ** 2 / (len(z) / 1024)).sum())
    assert scipy_stats.chi2.sf(chi2, 1023) > 1e-4
    assert scipy_stats.kstest(z, "uniform").pvalue > 1e-4
    # the low bits below the two-word resolution are populated too
    frac = (z * 2.0**34) % 1.0
    assert scipy_stats.kstest(frac[z > 0.5], "uniform").pvalue > 1e-4
