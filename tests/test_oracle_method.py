"""Pins for the oracle's PRNGD arithmetic (CPU only).

Each test checks the oracle against something the paper or the mathematics
fixes, not against a retyped copy of its own formula:

* Section 2, discrete degeneration: only x1 = a0 and x1 = a are rejected, so
  exhaustive enumeration at w = 8 rejects exactly 2 * 2^8 of 2^16 pairs.
* Eq. (3): every accepted z = x1 + k x2 lies in [a0 + k b, a + k b0].
* Uniformity ("strictly preserved", Section 1): at w = 8 the accepted pairs
  hit every value of the output grid exactly once, in increasing order of z.
* Eq. (5)/(6) endpoints: x1 = a0 + k, x2 = b0 maps to 0 and x1 = a - k,
  x2 = b maps to 1 - k^2 (rounded), never to 1.
* Eq. (5)/(6) in closed form: every output is within the rounding bound of
  the exact rational (1 - k^2) N / D, computed with Python fractions.
* The folded constant is the correctly rounded (1 - k^2) / D.
* Chi-square and Kolmogorov-Smirnov on 2^24 outputs (the method's premise:
  uniform output from independent uniform inputs, Section 2, last part).
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O

ONE_MINUS_ULP = float.fromhex("0x1.fffffffffffffp-1")


def exact_z(w, a0, a, b0, b, x1, x2):
    """Eq. (5) as an exact rational in the paper's own scale: every PRN is
    a multiple of k in [0, 1), trunc taken literally."""
    k = Fraction(1, 2**w)
    X1, X2, A0, A, B0, B = (Fraction(v) * k for v in (x1, x2, a0, a, b0, b))
    num = math.trunc((X1 - A0 - k) / k) + X2 - B0
    den = math.trunc((A - A0 - 2 * k) / k) + B - B0
    return num / den * (1 - k * k)


def ulp(x):
    return math.ulp(x) if x != 0 else math.ulp(0.0)


# ---------------------------------------------------------------- constant

RANGES = [
    # (w, a0, a, b0, b)
    (2, 0, 3, 0, 3), (3, 0, 7, 0, 7), (8, 0, 255, 0, 255), (8, 3, 200, 1, 250),
    (12, 0, 4095, 0, 4095), (16, 0, 65535, 0, 65535), (24, 0, 2**24 - 1, 0, 2**24 - 1),
    (26, 0, 2**26 - 1, 0, 2**26 - 1), (27, 0, 2**27 - 1, 0, 2**27 - 1),
    (32, 0, 2**32 - 1, 0, 2**32 - 1), (32, 1, O.M1, 1, O.M1), (32, 0, 2**32 - 1, 1, O.M1),
    (32, 17, 2**32 - 9, 5, 2**31), (20, 100, 900000, 7, 1000),
    # D = 1923 = 3 * 641 divides 2^64 - 1 with a 54-bit odd quotient: the
    # folded constant is an exact rounding tie (half-even decides it)
    (32, 0, 2, 0, 1923), (32, 5, 7, 10, 10 + 1923 * 2**9),
]


def test_degenerate_ranges_are_invalid():
    for ranges in [(0, 1, 0, 5), (0, 5, 3, 3), (0, 2**8, 0, 5), (0, 200, 0, 256)]:
        with pytest.raises(ValueError):
            O.PRNGD(None, 8, ranges=ranges)


@pytest.mark.parametrize("w,a0,a,b0,b", RANGES)
def test_scale_is_correctly_rounded(w, a0, a, b0, b):
    s = O.PRNGD(None, w, ranges=(a0, a, b0, b))
    k = Fraction(1, 2**w)
    D = (a - a0 - 2) * 2**w + (b - b0)
    assert s.D == D
    # Python converts a Fraction to float with correct rounding
    assert s.S == float((1 - k * k) / D)


def test_scale_values_for_the_standard_generators():
    # single generator on [0, 2^w - 1]: D = (2^w - 2) 2^w - 1, Eq. (6)
    for w in (2, 8, 16, 24, 32):
        s = O.PRNGD(O.GEN_PHILOX, w)
        assert s.D == (2**w - 2) * 2**w - 1
    assert O.PRNGD(O.GEN_MIXED, 32).D == (2**32 - 3) * 2**32 + (O.M1 - 1)
    assert O.PRNGD(O.GEN_MRG32K3A, 32).D == (O.M1 - 3) * 2**32 + (O.M1 - 1)


# -------------------------------------------------------- accept / reject

def test_exhaustive_w8_rejects_exactly_boundary_x1():
    s = O.PRNGD(O.GEN_ENUMERATE, 8)
    rejected = 0
    for p in range(2**16):
        x1, x2 = s.pair(p)
        assert (x1, x2) == (p >> 8, p & 255)
        acc = s.accept(x1)
        assert acc == (x1 not in (0, 255))
        rejected += not acc
    assert rejected == 512                       # fraction 2 / 2^8
    assert Fraction(rejected, 2**16) == Fraction(2, 2**8)


@pytest.mark.parametrize("w", [2, 3, 5, 10])
def test_rejection_fraction_is_two_over_two_to_w(w):
    s = O.PRNGD(O.GEN_ENUMERATE, w)
    total = 2**(2 * w)
    n_acc = (2**w - 2) * 2**w
    out, idx = s.fill(n_acc, with_index=True)
    # all accepted pairs of the full enumeration are consumed by the
    # last one, pair index 2^2w - 2^w - 1; the remaining 2^w pairs have
    # x1 = 2^w - 1 and are all rejected
    assert int(idx[-1]) == total - 2**w - 1
    assert Fraction(total - n_acc, total) == Fraction(2, 2**w)


def test_rejection_intervals_general_ranges_brute_force():
    # Section 2: with x2 in [b0, b] the rejected x1 are those below
    # a0 + k(b - b0) or above a - k(b - b0); decided here with fractions
    rng = random.Random(3)
    for _ in range(40):
        w = rng.randrange(3, 33)
        a0 = rng.randrange(0, 2**w - 3)
        a = rng.randrange(a0 + 2, 2**w)
        b0 = rng.randrange(0, 2**w - 1)
        b = rng.randrange(b0 + 1, min(2**w, b0 + 2**w))
        s = O.PRNGD(None, w, ranges=(a0, a, b0, b))
        k = Fraction(1, 2**w)
        for x1 in {a0, a0 + 1, a - 1, a, rng.randrange(a0, a + 1)}:
            X1, A0, A = x1 * k, a0 * k, a * k
            width = (b - b0) * k * k               # k (b - b0) in paper scale
            rejected = X1 < A0 + width or X1 > A - width
            assert s.accept(x1) == (not rejected)
            assert s.accept(x1) == (x1 not in (a0, a))


def test_accepted_z_lies_in_eq3_interval_exhaustive_w8_general_range():
    a0, a, b0, b, w = 3, 200, 1, 250, 8
    s = O.PRNGD(None, w, ranges=(a0, a, b0, b))
    k = Fraction(1, 2**w)
    lo = a0 * k + k * (b * k)            # a0 + k b in paper scale
    hi = a * k + k * (b0 * k)            # a + k b0
    zs = []
    for x1 in range(a0, a + 1):
        for x2 in range(b0, b + 1):
            if not s.accept(x1):
                continue
            z = x1 * k + k * (x2 * k)
            assert lo <= z <= hi
            zs.append((z, s.map(x1, x2), x1, x2))
    zs.sort()
    outs = [t[1] for t in zs]
    # the map is increasing in z and hits 0 and 1 - k^2 at the ends
    assert all(u < v for u, v in zip(outs, outs[1:]))
    assert outs[0] == 0.0
    assert (zs[0][2], zs[0][3]) == (a0 + 1, b0)
    assert abs(outs[-1] - float(1 - k * k)) <= ulp(outs[-1])
    assert (zs[-1][2], zs[-1][3]) == (a - 1, b)


# -------------------------------------------------------- uniformity

def test_exhaustive_w8_every_grid_value_exactly_once():
    s = O.PRNGD(O.GEN_ENUMERATE, 8)
    n = (256 - 2) * 256                   # all accepted pairs of 2^16
    out, idx = s.fill(n, with_index=True)
    assert s.counter == 2**16 - 256       # pairs after the last acceptance are all x1 = 255
    # N = (x1 - 1) 2^8 + x2 runs over 0..D once, in order
    N = np.array([((int(p) >> 8) - 1) * 256 + (int(p) & 255) for p in idx])
    np.testing.assert_array_equal(N, np.arange(n))
    assert np.all(np.diff(out) > 0)       # distinct grid values, increasing
    assert out[0] == 0.0 and out[-1] < 1.0
    # spacing of the grid: consecutive values differ by (1 - k^2) / D
    step = (1 - 2.0**-16) / s.D
    # (each value carries at most 2 ulp <= 2^-52 of rounding)
    assert np.allclose(np.diff(out), step, rtol=0, atol=2.0**-50)


# ----------------------------------------------------------- the map

@pytest.mark.parametrize("w", [2, 8, 16, 24, 26, 27, 32])
def test_map_endpoints_single_generator(w):
    s = O.PRNGD(O.GEN_PHILOX, w)
    top = 2**w - 1
    assert s.map(1, 0) == 0.0                        # x1 = a0 + k, x2 = b0
    z = s.map(top - 1, top)                          # x1 = a - k, x2 = b
    target = 1 - Fraction(1, 2**(2 * w))
    if w <= 26:
        assert abs(Fraction(z) - target) <= Fraction(ulp(z))
        assert z < 1.0
    else:
        assert z == ONE_MINUS_ULP                   # 1 - k^2 rounds to 1.0


def test_map_endpoints_mixed_and_mrg():
    for gen, a0 in ((O.GEN_MIXED, 0), (O.GEN_MRG32K3A, 1)):
        s = O.PRNGD(gen, 32)
        assert s.map(a0 + 1, 1) == 0.0
        assert s.map(a0 + 1, 2) == s.S
        _, a, _, b = s.ranges
        assert s.map(a - 1, b) == ONE_MINUS_ULP


def test_clamp_boundary_w32():
    # at w = 32 the products reach 1.0 only for x1 = 2^32 - 2 and the top
    # of x2; the result is then the largest double below 1
    s = O.PRNGD(O.GEN_PHILOX, 32)
    k2 = Fraction(1, 2**64)
    hits = 0
    for x2 in range(2**32 - 4096, 2**32):
        z = s.map(2**32 - 2, x2)
        assert z < 1.0
        N = (2**32 - 3) * 2**32 + x2
        unclamped = float(Fraction(float(N)) * Fraction(s.S))
        if unclamped >= 1.0:
            hits += 1
            assert z == ONE_MINUS_ULP
        else:
            assert z == unclamped
        # within the rounding bound of Eq. (6) either way
        assert abs(Fraction(z) - Fraction(N) * (1 - k2) / s.D) <= 3 * Fraction(ulp(z))
    assert hits == 1024


@pytest.mark.parametrize("w,a0,a,b0,b", RANGES)
def test_map_within_rounding_bound_of_eq5(w, a0, a, b0, b):
    """Three roundings (N to double, the constant, the product) give at most
    3 ulp; with N exact (2w <= 53) at most 2 ulp.  Almost all outputs are
    within 1 ulp of the correctly rounded exact value."""
    s = O.PRNGD(None, w, ranges=(a0, a, b0, b))
    rng = random.Random(w * 1000 + a0)
    bound = 2 if 2 * w <= 53 else 3
    near = 0
    trials = 400
    for _ in range(trials):
        x1 = rng.randrange(a0 + 1, a)
        x2 = rng.randrange(b0, b + 1)
        z = s.map(x1, x2)
        ex = exact_z(w, a0, a, b0, b, x1, x2)
        assert 0.0 <= z < 1.0
        if z == ONE_MINUS_ULP and ex >= Fraction(ONE_MINUS_ULP):
            near += 1
            continue
        assert abs(Fraction(z) - ex) <= bound * Fraction(ulp(z)), (x1, x2)
        near += abs(z - float(ex)) <= ulp(float(ex))
    assert near >= 0.99 * trials


def test_map_exact_integer_grid_small_w():
    # for 2w <= 53 N is exact, so the output is the product of two doubles
    # rounded once: it must equal the double nearest to N * S exactly
    for w in (4, 8, 12, 20, 26):
        s = O.PRNGD(O.GEN_PHILOX, w)
        rng = random.Random(w)
        for _ in range(300):
            x1 = rng.randrange(1, 2**w - 1)
            x2 = rng.randrange(0, 2**w)
            N = (x1 - 1) * 2**w + x2
            assert s.map(x1, x2) == float(Fraction(N) * Fraction(s.S))


# ------------------------------------------------------------ fill

def test_fill_concatenates_and_tracks_counter():
    for gen, w in ((O.GEN_PHILOX, 8), (O.GEN_PHILOX, 32), (O.GEN_MIXED, 32),
                   (O.GEN_MRG32K3A, 32), (O.GEN_ENUMERATE, 6)):
        whole = O.PRNGD(gen, w, seed=9, stream=4, counter=11)
        a, ia = whole.fill(3000, with_index=True)
        parts = O.PRNGD(gen, w, seed=9, stream=4, counter=11)
        b1, i1 = parts.fill(1234, with_index=True)
        b2, i2 = parts.fill(3000 - 1234, with_index=True)
        np.testing.assert_array_equal(a, np.concatenate([b1, b2]))
        np.testing.assert_array_equal(ia, np.concatenate([i1, i2]))
        assert whole.counter == parts.counter == int(ia[-1]) + 1


def test_fill_matches_pairwise_definition():
    for gen, w in ((O.GEN_PHILOX, 5), (O.GEN_MIXED, 32), (O.GEN_MRG32K3A, 32)):
        s = O.PRNGD(gen, w, seed=123, stream=2, counter=7)
        out, idx = s.fill(200, with_index=True)
        ref = O.PRNGD(gen, w, seed=123, stream=2)
        expect, pidx = [], []
        p = 7
        while len(expect) < 200:
            x1, x2 = ref.pair(p)
            if x1 not in ref.ranges[:2]:
                expect.append(ref.map(x1, x2))
                pidx.append(p)
            p += 1
        np.testing.assert_array_equal(out, np.array(expect))
        np.testing.assert_array_equal(idx, np.array(pidx, dtype=np.uint64))


def test_fill_w8_stream_has_binomial_rejections():
    s = O.PRNGD(O.GEN_PHILOX, 8, seed=42)
    n = 1 << 18
    s.fill(n)
    rejected = s.counter - n
    expect = n * (2 / 256) / (1 - 2 / 256)
    assert abs(rejected - expect) < 5 * math.sqrt(expect)


# ------------------------------------------------------------ statistics

@pytest.mark.parametrize("gen,w,seed", [(O.GEN_PHILOX, 32, 42), (O.GEN_MIXED, 32, 42),
                                        (O.GEN_PHILOX, 24, 7)])
def test_uniformity_chi2_and_ks_2_24_samples(gen, w, seed):
    s = O.PRNGD(gen, w, seed=seed)
    z = s.fill(1 << 24)
    assert z.min() >= 0.0 and z.max() < 1.0
    counts = np.bincount((z * 65536).astype(np.int64), minlength=65536)
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-4
    # the low half: the x2 contribution, frac(z 2^w), in 2^10 bins
    low = np.modf(z * 2.0**w)[0]
    counts_low = np.bincount((low * 1024).astype(np.int64), minlength=1024)
    assert stats.chisquare(counts_low).pvalue > 1e-4
    ks = stats.kstest(z, "uniform")
    assert ks.pvalue > 1e-4


# ------------------------------------------------------ map variants
# Eq. (4) -- Algorithm 1's Z -- maps the accepted region onto the open
# interval (0, 1); the last part of Section 2 suggests 1 - z' where zero
# must not occur.  Both are pinned against the paper's own formulas in
# exact rationals, not against the oracle's integer rewriting.

def algorithm1_z(w, a0, a, x1, x2):
    """Algorithm 1's Z for a single generator on [min, max] = [a0, a] k,
    R1 = x1 k, R2 = x2 k, in exact rationals."""
    k = Fraction(1, 2**w)
    R1, R2, mn, mx = Fraction(x1) * k, Fraction(x2) * k, Fraction(a0) * k, Fraction(a) * k
    return (R1 + k * R2 - (mn + k * mx)) / ((mx - mn) * (1 - k))


def eq4_z(w, a0, a, b0, b, x1, x2):
    """Eq. (4) in the paper's scale, exact rationals."""
    k = Fraction(1, 2**w)
    X1, X2, A0, A, B0, B = (Fraction(v) * k for v in (x1, x2, a0, a, b0, b))
    return (X1 + k * X2 - (A0 + k * B)) / (A - A0 - k * (B - B0))


def test_algorithm1_z_is_eq4_for_a_single_generator():
    rng = random.Random(41)
    for w in (3, 8, 16, 24, 32):
        a0, a = 0, 2**w - 1
        for _ in range(50):
            x1, x2 = rng.randrange(a0 + 1, a), rng.randrange(a0, a + 1)
            assert algorithm1_z(w, a0, a, x1, x2) == eq4_z(w, a0, a, a0, a, x1, x2)


@pytest.mark.parametrize("w,a0,a,b0,b", RANGES)
def test_eq4_map_within_rounding_bound(w, a0, a, b0, b):
    s = O.PRNGD(None, w, ranges=(a0, a, b0, b), map=O.MAP_EQ4)
    assert s.S4 == float(1 / Fraction(s.D4))         # the folded constant, correctly rounded
    rng = random.Random(w * 77 + a)
    bound = 2 if 2 * w <= 53 else 3
    near = 0
    trials = 400
    for _ in range(trials):
        x1 = rng.randrange(a0 + 1, a)
        x2 = rng.randrange(b0, b + 1)
        z = s.map(x1, x2)
        ex = eq4_z(w, a0, a, b0, b, x1, x2)
        assert 0 < ex < 1 and 0.0 < z < 1.0
        if z == ONE_MINUS_ULP and ex >= Fraction(ONE_MINUS_ULP):
            near += 1
            continue
        assert abs(Fraction(z) - ex) <= bound * Fraction(ulp(z)), (x1, x2)
        near += abs(z - float(ex)) <= ulp(float(ex))
    assert near >= 0.99 * trials


def test_eq4_exhaustive_w8_open_interval_increasing():
    s = O.PRNGD(O.GEN_ENUMERATE, 8, map=O.MAP_EQ4)
    out, idx = s.fill((256 - 2) * 256, with_index=True)
    assert np.all(np.diff(out) > 0)                  # distinct, in pair order
    assert out[0] > 0.0 and out[-1] < 1.0            # open at both ends
    # Algorithm 1's Z at the end points: (N + 1) / (D + 2) for the full range
    assert abs(Fraction(out[0]) - Fraction(1, s.D + 2)) <= Fraction(ulp(out[0]))
    assert abs(Fraction(out[-1]) - Fraction(s.D + 1, s.D + 2)) <= Fraction(ulp(out[-1]))


def test_eq4_top_clamps_at_w32():
    s = O.PRNGD(O.GEN_PHILOX, 32, map=O.MAP_EQ4)
    assert s.map(1, 0) > 0.0
    assert s.map(2**32 - 2, 2**32 - 1) == ONE_MINUS_ULP   # (D + 1) / (D + 2) rounds to 1


def test_one_minus_map_has_no_zero_and_reaches_one():
    s5 = O.PRNGD(O.GEN_ENUMERATE, 8)
    s1 = O.PRNGD(O.GEN_ENUMERATE, 8, map=O.MAP_ONE_MINUS)
    n = (256 - 2) * 256
    z5, z1 = s5.fill(n), s1.fill(n)
    assert np.all(z1 > 0.0) and np.all(z1 <= 1.0)
    assert z1[0] == 1.0                               # z' = 0 becomes 1
    assert np.all(np.diff(z1) < 0)                    # order reversed, values distinct
    # 1 - z' is a single rounding of the exact difference, and exact for
    # z' >= 1/2 (the difference of two doubles within a factor 2)
    for a, b in zip(z5[::97], z1[::97]):
        exact = 1 - Fraction(a)
        assert abs(Fraction(b) - exact) <= Fraction(ulp(b)) / 2
        if a >= 0.5:
            assert Fraction(b) == exact
    top = O.PRNGD(O.GEN_PHILOX, 32, map=O.MAP_ONE_MINUS).map(2**32 - 2, 2**32 - 1)
    assert top == 2.0**-53                            # the clamped 1 - 2^-53 turned over


# ------------------------------------ Algorithm 1's single-word consumption

def redraw_reference(words, A0, A, B0, B, w, count):
    """The one-word redraw built from the method's definition, in units of
    k = 2^-w (a word X stands for x = X k): the rejection intervals of
    Section 2 -- x1 < a0 + k (b - b0) or x1 > a - k (b - b0) -- tested on
    each first word in exact integers, the next word taken as x2, and each
    accepted pair mapped by Eq. (4) in exact rationals:
    z' = (x1 + k x2 - (a0 + k b)) / (a - a0 - k (b - b0)).  Returns the
    outputs and the number of words consumed.  The same interval test in
    FP64 (the precision the paper computes in) must decide alike."""
    two_w = 2**w
    k = 2.0**-w
    lo_dp = A0 * k + k * ((B - B0) * k)
    hi_dp = A * k - k * ((B - B0) * k)
    den = (A - A0) * two_w - (B - B0)
    it = iter(words)
    used, out = 0, []
    while len(out) < count:
        X1 = next(it)
        used += 1
        rejected = X1 * two_w < A0 * two_w + (B - B0) or X1 * two_w > A * two_w - (B - B0)
        assert rejected == (X1 * k < lo_dp or X1 * k > hi_dp)
        if rejected:
            continue
        X2 = next(it)
        used += 1
        out.append(Fraction((X1 - A0) * two_w + X2 - B, den))
    return out, used


def _philox_w_words(seed, stream, count, w):
    return [int(u) >> (32 - w) for u in O.philox_words(seed, stream, 0, count)]


@pytest.mark.parametrize("w,seed", [(3, 1), (5, 2), (8, 3), (12, 4), (16, 5)])
def test_single_consumption_is_the_one_word_redraw(w, seed):
    n = 3000
    words = _philox_w_words(seed, 0, 4 * n + 64, w)
    Z, calls = redraw_reference(words, 0, 2**w - 1, 0, 2**w - 1, w, n)
    s = O.PRNGD(O.GEN_PHILOX, w, seed=seed, map=O.MAP_EQ4, consume=O.CONSUME_SINGLE)
    out = s.fill(n)
    assert s.counter == calls                        # the same words consumed
    bound = 2 if 2 * w <= 53 else 3
    for z, ex in zip(out, Z):
        assert 0.0 < z < 1.0
        assert abs(Fraction(z) - ex) <= bound * Fraction(ulp(z))


def test_single_consumption_mrg32k3a_is_the_one_word_redraw():
    n = 2000
    state = O.mrg_stream_base(7, 0)
    outs, _ = O.mrg_outputs(state, 2 * n + 16)
    words = [int(v) for v in outs]
    Z, calls = redraw_reference(words, 1, O.M1, 1, O.M1, 32, n)
    s = O.PRNGD(O.GEN_MRG32K3A, 32, seed=7, map=O.MAP_EQ4, consume=O.CONSUME_SINGLE)
    out = s.fill(n)
    assert s.counter == calls == 2 * n               # no rejection this early
    for z, ex in zip(out, Z):
        assert abs(Fraction(z) - ex) <= 3 * Fraction(ulp(z))


def test_single_and_pair_consumption_agree_until_the_first_rejection():
    w = 8
    pair = O.PRNGD(O.GEN_PHILOX, w, seed=9)
    single = O.PRNGD(O.GEN_PHILOX, w, seed=9, consume=O.CONSUME_SINGLE)
    zp, idx = pair.fill(400, with_index=True)
    zs = single.fill(400)
    # the first rejected pair index is the first gap in the accepted indices
    gaps = np.flatnonzero(np.diff(idx.astype(np.int64)) != 1)
    first = int(gaps[0]) + 1 if idx[0] == 0 else 0
    assert first > 0
    np.testing.assert_array_equal(zp[:first], zs[:first])
    # after it, single consumption is realigned by one word: the next output
    # pairs the word after the rejected x1 with the one after it
    rej_word = 2 * (int(idx[first - 1]) + 1)
    x1, x2 = single.word(rej_word + 1), single.word(rej_word + 2)
    if pair.accept(x1):
        assert zs[first] == pair.map(x1, x2)


def test_single_consumption_refuses_two_generators():
    with pytest.raises(ValueError):
        O.PRNGD(O.GEN_MIXED, 32, consume=O.CONSUME_SINGLE)
