"""The oracle walked in pieces: the accepted pairs of consecutive pair
ranges, concatenated, are the sequential fill (Section 2: pairs are taken
one after another, and a pair's fate depends on that pair alone), so a
long stream may be spread over host cores for full-size comparisons."""
import numpy as np
import pytest

import oracle as O
import oracle_parallel as OP


@pytest.mark.parametrize("gen,w,counter,n", [
    (O.GEN_PHILOX, 3, 5, 60000), (O.GEN_PHILOX, 32, 1, 200000), (O.GEN_PHILOX, 24, 0, 50000),
    (O.GEN_MIXED, 32, 7, 30000), (O.GEN_MRG32K3A, 32, 3, 30000),
    (O.GEN_ENUMERATE, 4, 9, 5000), (O.GEN_PHILOX, 8, 2**64 - 2**17, 100000)])
def test_pieces_concatenate_to_the_sequential_fill(gen, w, counter, n):
    ref = O.PRNGD(gen, w, seed=9, stream=4, counter=counter)
    expect = ref.fill(n)
    for chunk in (1, 2, 997, 10007):
        if chunk == 1 and n > 5000:
            continue
        got, end = OP.fill_long(gen, w, 9, 4, counter, n, threads=4, chunk_pairs=chunk)
        assert np.array_equal(got.view(np.uint64), expect.view(np.uint64)), chunk
        assert end == ref.counter, chunk


def test_fill_pairs_examines_exactly_its_range():
    # w = 3: a quarter of the pairs are rejected; every pair of the range is
    # examined once, and the count matches a brute-force walk over pairs
    s = O.PRNGD(O.GEN_PHILOX, 3, seed=1, counter=100)
    vals = s.fill_pairs(1100, 1000)
    assert s.counter == 1100
    kept = [p for p in range(100, 1100) if s.accept(s.pair(p)[0])]
    assert len(vals) == len(kept)
    assert np.array_equal(vals, [s.map(*s.pair(p)) for p in kept])
    # a cap on the outputs stops the walk right after the last one it made
    t = O.PRNGD(O.GEN_PHILOX, 3, seed=1, counter=100)
    part = t.fill_pairs(1100, 10)
    assert np.array_equal(part, vals[:10]) and t.counter == kept[9] + 1


def test_independent_streams_in_parallel():
    specs = [(s * 7 + 1, s, 3 * s, 1000 + s) for s in range(20)]
    outs, ctrs = OP.fill_streams(O.GEN_PHILOX, 8, specs, threads=4)
    for (seed, st, c, n), o, e in zip(specs, outs, ctrs):
        r = O.PRNGD(O.GEN_PHILOX, 8, seed=seed, stream=st, counter=c)
        assert np.array_equal(o, r.fill(n)) and e == r.counter
