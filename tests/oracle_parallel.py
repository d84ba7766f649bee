"""The oracle spread over host cores, for full-size comparisons (test
infrastructure).

Independent streams run one per task.  One long stream is walked as
consecutive pair ranges, each on its own thread: the accepted pairs of
[c, e) followed by those of [e, f) are the accepted pairs of [c, f), so the
concatenation is the sequential fill.  The oracle's C calls release the
interpreter lock, so threads run in parallel.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def host_threads(cap=16):
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def fill_streams(gen, w, specs, threads=None, map=O.MAP_EQ5, arity=2):
    """specs: [(seed, stream, counter, n), ...].  Returns (outputs, counters):
    a list of float64 arrays and the counter after each, in order."""
    def one(spec):
        seed, stream, counter, n = spec
        s = O.PRNGD(gen, w, seed=seed, stream=stream, counter=counter, map=map, arity=arity)
        return s.fill(n), s.counter

    with ThreadPoolExecutor(max_workers=threads or host_threads()) as pool:
        res = list(pool.map(one, specs))
    return [r[0] for r in res], [r[1] for r in res]


def fill_long(gen, w, seed, stream, counter, n, threads=None, chunk_pairs=1 << 24, arity=2):
    """The first n outputs of one stream from pair (or triple) `counter`, and
    the counter after them, walked as consecutive ranges on several
    threads."""
    threads = threads or host_threads()
    out = np.empty(n, dtype=np.float64)
    top = (1 << 64) - 1

    def walk(start):
        end = min(start + chunk_pairs, top)
        s = O.PRNGD(gen, w, seed=seed, stream=stream, counter=start, arity=arity)
        return start, s.fill_pairs(end, end - start)

    made = 0
    start = counter
    with ThreadPoolExecutor(max_workers=threads) as pool:
        while made < n:
            if start >= top:
                raise ValueError("stream runs past the last pair")
            starts = []
            for _ in range(threads):
                if start >= top:
                    break
                starts.append(start)
                start = min(start + chunk_pairs, top)
            for first, vals in pool.map(walk, starts):
                if made >= n:
                    break
                take = min(len(vals), n - made)
                out[made:made + take] = vals[:take]
                made += take
                if made == n:
                    # the counter: walk this range again up to the n-th output
                    s = O.PRNGD(gen, w, seed=seed, stream=stream, counter=first,
                                arity=arity)
                    s.fill(take)
                    return out, s.counter
    raise AssertionError("unreachable")
