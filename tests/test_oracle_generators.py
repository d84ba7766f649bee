"""Pins for the oracle's base generators (CPU only).

Philox4x32-10 and MRG32k3a are checked against an independent library
(rocRAND, built from its source headers for the host), and MRG32k3a also
against properties fixed by its definition: one-step recurrence versus
matrix jump-ahead, and the full-period identity A^(m^3 - 1) = I that a
wrong multiplier or modulus breaks.
"""
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
XCHECK_SRC = os.path.join(HERE, "xcheck", "rocrand_xcheck.cpp")
XCHECK_BIN = os.path.join(HERE, "xcheck", "_build", "rocrand_xcheck")


@pytest.fixture(scope="module")
def xcheck():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND cross-check")
    if (not os.path.exists(XCHECK_BIN)
            or os.path.getmtime(XCHECK_BIN) < os.path.getmtime(XCHECK_SRC)):
        os.makedirs(os.path.dirname(XCHECK_BIN), exist_ok=True)
        # build under a private name, then rename: parallel test workers
        # may build at the same time
        tmp = f"{XCHECK_BIN}.{os.getpid()}"
        subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1",
                        XCHECK_SRC, "-o", tmp], check=True)
        os.replace(tmp, XCHECK_BIN)

    def run(*args):
        out = subprocess.run([XCHECK_BIN, *map(str, args)], check=True,
                             capture_output=True, text=True).stdout
        return np.array([int(v) for v in out.split()], dtype=np.uint64)
    return run


# ---------------------------------------------------------------- Philox

PHILOX_CASES = [
    # (seed, stream, first word, count)
    (42, 0, 0, 64),
    (42, 7, 1000, 33),
    (0, 0, 0, 16),
    (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, 12345, 20),
    (0x0123456789ABCDEF, 65535, 4 * (2**32 - 2), 24),   # block c0 -> c1 carry
    (99, 3, 4 * (2**62 - 3), 12),                         # last word indices
]


@pytest.mark.parametrize("seed,stream,first,count", PHILOX_CASES)
def test_philox_words_match_rocrand(xcheck, seed, stream, first, count):
    ours = O.philox_words(seed, stream, first, count).astype(np.uint64)
    # rocRAND: key = seed, counter words (2,3) = subsequence, word offset
    theirs = xcheck("philox", seed, stream << 32, first, count)
    np.testing.assert_array_equal(ours, theirs)


def test_philox_pairs_near_top_of_pair_counter(xcheck):
    # the largest pair counters (2^64 - 1) use words near 2^65, which
    # rocRAND reaches with two word skips of p0 each
    s = O.PRNGD(O.GEN_PHILOX, 32, seed=77, stream=5)
    p0 = 2**64 - 6
    pairs = [s.pair(p) for p in range(p0, p0 + 6)]
    words = xcheck("philox", 77, 5 << 32, p0, 12, p0)
    np.testing.assert_array_equal(np.array(pairs, dtype=np.uint64).ravel(), words)


def test_philox_block_function_counter_layout():
    # word j of a stream is lane j mod 4 of block j / 4 with counter
    # (block lo, block hi, 0, stream): check the layout through the block
    # function itself at a block index that carries into the high word
    block = 2**32 + 5
    words = O.philox_words(7, 9, 4 * block, 4)
    direct = O.philox4x32_10([block & 0xFFFFFFFF, block >> 32, 0, 9], [7, 0])
    np.testing.assert_array_equal(words, direct)


# ------------------------------------------------------------- MRG32k3a

def test_mrg_first_outputs_match_rocrand(xcheck):
    ours, _ = O.mrg_outputs([12345] * 6, 100)
    theirs = xcheck("mrg", *([12345] * 6), 0, 0, 0, 100)
    np.testing.assert_array_equal(ours.astype(np.uint64), theirs)


@pytest.mark.parametrize("seed,stream,offset", [
    (0, 0, 0), (0, 1, 0), (1, 0, 0), (42, 0, 0), (42, 3, 17),
    (2**64 - 1, 2**32 - 1, 2**63 + 11), (12345, 65535, 2**40 + 3),
])
def test_mrg_streams_match_rocrand_jumps(xcheck, seed, stream, offset):
    base = O.mrg_stream_base(seed, stream)
    st = O.mrg_jump(base, offset)
    ours, _ = O.mrg_outputs(st, 40)
    theirs = xcheck("mrg", *([12345] * 6), seed, stream, offset, 40)
    np.testing.assert_array_equal(ours.astype(np.uint64), theirs)


def test_mrg_outputs_in_range():
    out, _ = O.mrg_outputs([12345] * 6, 200000)
    assert out.min() >= 1 and out.max() <= O.M1


def test_mrg_jump_equals_stepping():
    rng = random.Random(5)
    for _ in range(20):
        st0 = [rng.randrange(1, O.M1) for _ in range(3)] + \
              [rng.randrange(1, O.M2) for _ in range(3)]
        e = rng.randrange(0, 5000)
        _, stepped = O.mrg_outputs(st0, e)
        jumped = O.mrg_jump(st0, e)
        np.testing.assert_array_equal(stepped, jumped)


def test_mrg_jump_composes():
    rng = random.Random(6)
    st0 = [12345] * 6
    for _ in range(10):
        e1 = rng.randrange(0, 2**130)
        e2 = rng.randrange(0, 2**60)
        np.testing.assert_array_equal(O.mrg_jump(O.mrg_jump(st0, e1), e2),
                                      O.mrg_jump(st0, e1 + e2))


@pytest.mark.parametrize("component,m", [(0, O.M1), (1, O.M2)])
def test_mrg_full_period_identity(component, m):
    eye = np.eye(3, dtype=np.uint64)
    np.testing.assert_array_equal(O.mrg_matpow(component, m**3 - 1), eye)
    # and the one-step matrix is not the identity at a few short periods
    for e in (1, 2, 3, m - 1, m + 1, m**2 - 1):
        assert not np.array_equal(O.mrg_matpow(component, e), eye)
