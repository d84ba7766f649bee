"""A CPU model of the speculative fill and its repair rules.

The speculative kernels store each tile at the offset its hint gives (the
rejections of earlier tiles of its segment published so far), and a repair
pass then redoes exactly the tiles that (a) assumed too few earlier
rejections, (b) may hold stale values written there by an earlier tile, or
(c) hold output n - 1.  This model replays those rules with random
rejection patterns, random tile execution orders, random hint visibility
and the racing writes of the next pair counter, and checks that the final
outputs and counter equal the sequential definition.  Outputs are modelled
as pair indices, so any misplaced value is caught.
"""
import random

import pytest


def simulate(n, lo0, T, p, seed):
    rnd = random.Random(seed)
    # planned tiles: like planned_pairs with slack 0..2 tiles
    planned = n + rnd.randint(0, 3)
    ntiles = max(1, -(-(planned + lo0) // T))  # windows covering [lo0, lo0+planned)
    # acceptance per pair index (pair index relative to window 0 start)
    maxpairs = (ntiles + 50) * T + 10 * n + 1000
    acc = [rnd.random() >= p for _ in range(maxpairs)]
    # truth
    truth = []
    q = lo0
    while len(truth) < n:
        if acc[q]:
            truth.append(q)
        q += 1
    true_counter = truth[-1] + 1
    out = [None] * n
    counter = [None]
    def window(w, lo_off):
        return [q for q in range(w * T + lo_off, (w + 1) * T) if acc[q]]
    def run(w, lo_off, excl, spec):
        left = n - excl
        kept = window(w, lo_off)
        clean = lo_off == 0 and len(kept) == T
        if spec and lo_off == 0:
            lim = T if left > T else left
            for qq in range(lim):
                out[excl + qq] = ('spec', w * T + qq)
            if left <= T:
                # the spec pass writes the counter before knowing the window is clean
                counter[0] = w * T + left
        if not (spec and clean):
            for r, pq in enumerate(kept):
                if r < left:
                    out[excl + r] = pq
                if r + 1 == left:
                    counter[0] = pq + 1
        else:
            # clean spec: values are right: replace markers by pair ids
            lim = T if left > T else left
            for qq in range(lim):
                out[excl + qq] = w * T + qq
        return len(kept)
    entries = []          # (tile, rej) in append order
    hint = [0] * ntiles
    order = list(range(ntiles))
    rnd.shuffle(order)
    visible = set()
    for idx, t in enumerate(order):
        # hint: entries visible of tiles < t
        used = sum(r for (et, r) in entries if et < t and rnd.random() < 0.7) if t > 0 else 0
        hint[t] = used
        lo = lo0 if t == 0 else 0
        excl = (0 if t == 0 else t * T - lo0) - used
        w = t
        if excl < n:
            kept = run(w, lo, excl, True)
        else:
            kept = len(window(w, lo))
        rej = (T - lo) - kept
        if rej:
            entries.append((t, rej))
        if t == ntiles - 1:
            running = excl + kept
            w2 = w + 1
            while running < n:
                running += run(w2, 0, running, True)
                w2 += 1
    # repair
    def facts(g):
        P = sum(r for (et, r) in entries if et < g)
        rej = sum(r for (et, r) in entries if et == g)
        after = any(et < g for (et, r) in entries)
        return P, rej, after
    redo = []
    for g in range(1, ntiles):
        P, rej, after = facts(g)
        if not after:
            continue
        off = g * T - lo0 - P
        if off >= n:
            continue
        need = False
        if hint[g] != P:
            need = True
        elif off + (T - rej) >= n or g == ntiles - 1:
            need = True
        else:
            gap = 0
            v = g - 1
            while True:
                Pv, rv, av = facts(v)
                reach = (Pv - hint[v]) + rv
                if reach > gap:
                    need = True
                    break
                if not av or v == 0:
                    break
                gap += T - (lo0 if v == 0 else 0) - rv
                if gap >= P + T:
                    break
                v -= 1
        if need:
            redo.append((g, off))
    rnd.shuffle(redo)
    for g, off in redo:
        running = off + run(g, 0, off, False)
        if g == ntiles - 1:
            w2 = g + 1
            while running < n:
                running += run(w2, 0, running, True)
                w2 += 1
    ok = out == truth and counter[0] == true_counter
    return ok, len(entries), len(redo)



@pytest.mark.parametrize("block", range(8))
def test_repair_rules_leave_the_sequential_outputs(block):
    for seed in range(block * 400, (block + 1) * 400):
        rnd = random.Random(seed * 7 + 1)
        T = rnd.choice([4, 8, 16])
        n = rnd.randint(1, 12 * T)
        lo0 = rnd.randint(0, T - 1)
        p = rnd.choice([0.0, 0.01, 0.05, 0.2, 0.5])
        ok, entries, redone = simulate(n, lo0, T, p, seed)
        assert ok, (seed, T, n, lo0, p, entries, redone)
