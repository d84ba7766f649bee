"""A CPU model of the chunk-speculative batch fill and its repair.

The chunk kernel takes each request (segment) in chunks of P pairs, chunk
k of a segment starting at pair w0 P + k P of its stream (the first one
lo0 pairs in).  Chunk k stores at the offset it would have if no earlier
chunk of its segment rejected a pair (k P - lo0; 0 for k = 0).  A chunk
whose P outputs all lie below output n - 1 stores all P pair values at
once, as if it rejected nothing, and checks afterwards; any other chunk is
produced exactly (ranks), writing the next position when it holds output
n - 1, and counts as clean when its accepted pairs up to output n - 1 leave
no later chunk an output.  A chunk that is not clean marks its segment
dirty from its index (the smallest index wins).  The last planned chunk, if
clean, takes every further chunk until n outputs.  Then the repair
produces every dirty segment again, exactly and in order, from its first
dirty chunk, writing the next position last.

The model replays these rules with random rejection patterns, random
chunk execution orders (stores of different chunks land in any order), and
checks that the final outputs (modelled as pair indices, so any misplaced
or stale value is caught) and next positions equal the sequential
definition, and that no chunk ever writes below its true offset or past
output n - 1.
"""
import random

import pytest


def chunk_fill(n, lo0, P, p, planned_extra, seed):
    rnd = random.Random(seed)
    planned = n + planned_extra
    ntiles = max(1, -(-(planned + lo0) // P))
    span = (ntiles + 64) * P + 20 * n + 4096
    acc = [rnd.random() >= p for _ in range(span)]
    truth, q = [], lo0
    while len(truth) < n:
        if acc[q]:
            truth.append(q)
        q += 1
    # true offset of each pair position's chunk start
    def true_offset(k):
        start = lo0 if k == 0 else k * P
        return sum(1 for x in range(lo0, start) if acc[x])

    out = [("unwritten",)] * n
    writes = []                       # (chunk, position) of every chunk-kernel store
    counter = []                      # next-position writes of the chunk kernel, in order
    first_dirty = None
    k_full = (n + lo0 - 1) // P
    k_end = (n + lo0 + P - 1) // P

    def exact(ch, lo_off, excl, log):
        """Pairs of chunk ch from offset lo_off at output excl; returns the
        kept count, or P - lo_off once output n - 1 is stored."""
        running = excl
        for x in range(ch * P + lo_off, (ch + 1) * P):
            if running >= n:
                return P - lo_off
            if acc[x]:
                log.append((running, x))
                if running + 1 == n:
                    log.append(("counter", x + 1))
                running += 1
        return running - excl if running < n else P - lo_off

    order = list(range(ntiles))
    rnd.shuffle(order)
    for k in order:
        if k >= k_end:
            continue
        lo_off = lo0 if k == 0 else 0
        excl = 0 if k == 0 else k * P - lo0
        log = []
        if lo_off == 0 and k < k_full:
            # store-first: every pair of the chunk, as if all were accepted
            assert excl + P < n
            for j in range(P):
                log.append((excl + j, k * P + j))
            clean = all(acc[k * P + j] for j in range(P))
        else:
            clean = exact(k, lo_off, excl, log) == P - lo_off
        if not clean:
            first_dirty = k if first_dirty is None else min(first_dirty, k)
        elif k == ntiles - 1:
            running = excl + (P - lo_off)
            c2 = k + 1
            while running < n:
                running += exact(c2, 0, running, log)
                c2 += 1
        for item in log:
            if item[0] == "counter":
                counter.append(item[1])
            else:
                pos, x = item
                assert 0 <= pos < n, "a chunk wrote outside the output"
                # never below the true offset of the chunk's first pair
                assert pos >= true_offset(k) - 0, "a chunk wrote below its true offset"
                writes.append((k, pos, x))
    # stores of different chunks land in any order: shuffle, keeping each
    # chunk's own order (a lane writes its position once per pass)
    rnd.shuffle(writes)
    for _, pos, x in writes:
        out[pos] = x
    final_counter = counter[-1] if counter else None
    if first_dirty is not None:
        k0 = first_dirty
        running = 0 if k0 == 0 else k0 * P - lo0
        assert running == true_offset(k0)
        ch = k0
        log = []
        while running < n:
            running += exact(ch, lo0 if ch == 0 else 0, running, log)
            ch += 1
        for item in log:
            if item[0] == "counter":
                final_counter = item[1]
            else:
                out[item[0]] = item[1]
    return out, final_counter, truth, truth[-1] + 1


@pytest.mark.parametrize("P", [128, 256, 512])
@pytest.mark.parametrize("p", [0.0, 1e-4, 0.003, 0.05, 0.4])
def test_chunk_form_equals_the_sequential_fill(P, p):
    rnd = random.Random(int(P * 1000 + p * 1e6))
    for trial in range(40):
        n = rnd.choice([1, 2, P - 1, P, P + 1, 2 * P - 1, 3 * P + 5, rnd.randint(1, 9 * P)])
        lo0 = rnd.choice([0, 1, P - 1, rnd.randrange(P)])
        extra = rnd.choice([0, 1, 3, P, 3 * P])
        out, ctr, truth, tctr = chunk_fill(n, lo0, P, p, extra, seed=trial * 7919 + n)
        assert out == truth, (P, p, trial, n, lo0, extra)
        assert ctr == tctr, (P, p, trial, n, lo0, extra)


def test_no_planned_slack_and_many_rejections():
    # the last planned chunk continues far past its own pairs
    for trial in range(30):
        out, ctr, truth, tctr = chunk_fill(3000, trial % 7, 128, 0.3, 0, seed=trial)
        assert out == truth and ctr == tctr


def counted_fill(n, lo0, P, p, planned_extra, seed, block=4):
    """The counted single fill: chunk k covers pairs [k P, (k + 1) P) of
    the stream's grid (chunk 0 from lo0); pass 1 counts each chunk's
    accepted pairs, a two-level scan (blocks of `block` chunks, then the
    block totals) gives exact offsets, pass 2 stores each chunk's accepted
    pairs below output n at its offset; the last chunk continues."""
    rnd = random.Random(seed)
    planned = n + planned_extra
    chunks = max(1, -(-planned // P))
    span = (chunks + 64) * P + 20 * n + 4096
    acc = [rnd.random() >= p for _ in range(span)]
    truth, q = [], lo0
    while len(truth) < n:
        if acc[q]:
            truth.append(q)
        q += 1
    lo = lambda k: lo0 if k == 0 else 0          # noqa: E731
    counts = [sum(acc[k * P + lo(k):(k + 1) * P]) for k in range(chunks)]
    nblocks = -(-chunks // block)
    local, totals = [0] * chunks, []
    for b in range(nblocks):
        run = 0
        for k in range(b * block, min(chunks, (b + 1) * block)):
            local[k] = run
            run += counts[k]
        totals.append(run)
    block_off = [sum(totals[:b]) for b in range(nblocks)]
    out, counter = [None] * n, None

    def produce(k, off):
        nonlocal counter
        for x in range(k * P + lo(k), (k + 1) * P):
            if acc[x]:
                if off < n:
                    out[off] = x
                    if off == n - 1:
                        counter = x + 1
                off += 1
        return off

    order = list(range(chunks))
    rnd.shuffle(order)
    for k in order:
        off = block_off[k // block] + local[k]
        end = produce(k, off) if off < n else off + counts[k]
        if k == chunks - 1:
            c2 = k + 1
            while end < n:
                end = produce(c2, end)
                c2 += 1
    return out, counter, truth, truth[-1] + 1


@pytest.mark.parametrize("p", [0.0, 1e-3, 0.05, 0.25, 0.6])
def test_counted_form_equals_the_sequential_fill(p):
    rnd = random.Random(int(p * 1e6) + 5)
    for trial in range(60):
        P = rnd.choice([8, 16, 512])
        n = rnd.choice([1, 2, P - 1, P, P + 1, 7 * P + 3, rnd.randint(1, 40 * P)])
        lo0 = rnd.choice([0, 1, P - 1, rnd.randrange(P)])
        extra = rnd.choice([0, 1, P, 5 * P])
        out, ctr, truth, tctr = counted_fill(n, lo0, P, p, extra, seed=trial * 31 + n)
        assert out == truth and ctr == tctr, (p, trial, P, n, lo0, extra)
