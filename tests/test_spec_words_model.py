"""A CPU model of the one-word-consumption fill across workgroups.

Under Algorithm 1's one-word redraw, word r of a fill is a *candidate* when
it equals a0 or a.  The speculative kernel lets every window of T words
(the first one starting lo0 <= c0 words before the fill's first word c0,
lo0 < T chosen freely) be produced by its own workgroup from a hint -- the rejected r1 it can infer
from the earlier windows' candidates published so far -- and a repair pass
then produces again exactly the windows that (a) took a hint below the
truth, (b) may hold values a wrong earlier window wrote past its true end,
or (c) hold output n - 1, or are the last window, behind a wrong one.

This model replays that with small windows, small w (so that candidates
are everywhere), random start positions and window origins, random hint
visibility and random window execution orders, and checks that the final outputs (modelled as
the word indices of each output's r1 and r2) and the final word position
equal Algorithm 1's sequential walk.  It also checks the two facts the
kernels rest on: a candidate is a rejected r1 exactly when its distance to
the previous candidate is odd, and a hint taken from any subset of the
earlier candidates never exceeds the truth.
"""
import random

import pytest


def sequential(words, a0, a, c0, n):
    """Algorithm 1's loop over the word stream: outputs as (r1, r2) word
    indices and the next word position."""
    out = []
    q = c0
    while len(out) < n:
        while words[q] in (a0, a):
            q += 1
        out.append((q, q + 1))
        q += 2
    return out, q


def skips_of(rs):
    """Rejected r1 among candidates at relative positions rs (any order),
    by the previous-candidate rule."""
    rs = sorted(rs)
    prev, k = -1, 0
    for r in rs:
        k += (r - prev) & 1
        prev = r
    return k


def walk_window(words, a0, a, c0, T, wb, lo, state, running, n, mem, counter):
    """Produce the window of words wb + lo .. wb + T - 1 from (state,
    running) exactly; writes outputs below n into mem and the counter for
    output n - 1.  Returns the state after the window."""
    for q in range(wb + lo, wb + T):
        if running >= n:
            break
        if state == 0:
            state = 0 if words[q] in (a0, a) else 1
        else:
            if running < n:
                mem[running] = (q - 1, q)
                if running == n - 1:
                    counter[0] = q + 1
            running += 1
            state = 0
    return state, running


def simulate(w, T, c0, n, seed, drop_rule=None):
    rnd = random.Random(seed)
    a0, a = 0, 2 ** w - 1
    total = c0 + 4 * n + 40 * T + 64
    words = [rnd.randrange(2 ** w) for _ in range(total)]
    truth, true_counter = sequential(words, a0, a, c0, n)
    lo0 = c0 % T if rnd.random() < 0.3 else rnd.randrange(0, min(c0, T - 1) + 1)
    wb0 = c0 - lo0   # the first window's first word
    planned_words = 2 * (n + rnd.randint(0, 3))
    ntiles = -(-planned_words // T) + 1

    # candidates per tile, as relative positions
    cands = {}
    for t in range(ntiles):
        lo = lo0 if t == 0 else 0
        for qq in range(lo, T):
            q = wb0 + t * T + qq
            if words[q] in (a0, a):
                cands.setdefault(t, []).append(q - c0)
    all_before = lambda t: [r for v in range(t) for r in cands.get(v, [])]

    mem = [None] * n
    counter = [None]
    hints = {}
    order = list(range(ntiles))
    rnd.shuffle(order)
    for t in order:
        earlier = all_before(t)
        vis = [r for r in earlier if rnd.random() < 0.5] if rnd.random() < 0.7 else earlier
        h = skips_of(vis)
        assert h <= skips_of(earlier)          # a hint never exceeds the truth
        hints[t] = h
        if t == 0:
            state, running = 0, 0
        else:
            done = t * T - lo0 - h
            state, running = done & 1, done >> 1
        lo = lo0 if t == 0 else 0
        state, running = walk_window(words, a0, a, c0, T, wb0 + t * T, lo, state, running, n,
                                     mem, counter)
        if t == ntiles - 1:
            w2 = wb0 + (t + 1) * T
            while running < n:
                state, running = walk_window(words, a0, a, c0, T, w2, 0, state, running, n, mem,
                                             counter)
                w2 += T

    # repair, from the complete list
    cnt = sum(len(v) for v in cands.values())

    def facts(g):
        before = all_before(g)
        allr = before + cands.get(g, [])
        h = skips_of(before)
        k = skips_of(allr) - h
        return h, len(cands.get(g, [])), k, bool(before)

    redo = []
    for g in range(1, ntiles):
        h, c, k, dirty = facts(g)
        if not dirty:
            continue
        r0 = g * T - lo0
        off = (r0 - h) >> 1
        if off >= n:
            continue
        if drop_rule != "a" and hints[g] != h:
            redo.append((g, h))
            continue
        off_end = (r0 + T - h - k) >> 1
        if off_end >= n or g == ntiles - 1:
            if drop_rule != "c":
                redo.append((g, h))
            continue
        if drop_rule == "b":
            continue
        gap, bound = 0, (cnt + 2) // 2
        v = g - 1
        while True:
            hv, cv, kv, dv = facts(v)
            reach = 0 if hints[v] == hv else (hv - hints[v] + cv + 2) // 2
            if reach > gap:
                redo.append((g, h))
                break
            if not dv:
                break
            rv = v * T - lo0
            gap += ((rv + T - hv - kv) >> 1) - ((rv - hv) >> 1)
            if gap >= bound:
                break
            v -= 1
    rnd.shuffle(redo)
    for g, h in redo:
        done = g * T - lo0 - h
        state, running = walk_window(words, a0, a, c0, T, wb0 + g * T, 0, done & 1, done >> 1,
                                     n, mem, counter)
        if g == ntiles - 1:
            w2 = wb0 + (g + 1) * T
            while running < n:
                state, running = walk_window(words, a0, a, c0, T, w2, 0, state, running, n,
                                             mem, counter)
                w2 += T
    return mem == truth and counter[0] == true_counter


def test_previous_candidate_rule_is_the_automaton():
    rnd = random.Random(3)
    for _ in range(300):
        w = rnd.choice([2, 3, 4])
        a0, a = 0, 2 ** w - 1
        words = [rnd.randrange(2 ** w) for _ in range(200)]
        state, skips = 0, []
        for r, x in enumerate(words):
            if state == 0:
                if x in (a0, a):
                    skips.append(r)
                else:
                    state = 1
            else:
                state = 0
        cands = [r for r, x in enumerate(words) if x in (a0, a)]
        prev, rule = -1, []
        for r in cands:
            if (r - prev) & 1:
                rule.append(r)
            prev = r
        assert rule == skips


@pytest.mark.parametrize("w", [2, 3, 5])
def test_speculative_words_fill_equals_the_sequential_walk(w):
    rnd = random.Random(w)
    for seed in range(150):
        T = rnd.choice([8, 16, 32])
        c0 = rnd.randrange(0, 5 * T)
        n = rnd.randrange(1, 12 * T)
        assert simulate(w, T, c0, n, seed * 7919 + w), (w, T, c0, n, seed)


@pytest.mark.parametrize("rule", ["a", "b", "c"])
def test_each_repair_rule_is_needed(rule):
    # without any one of the three rules some case ends wrong
    failures = 0
    for seed in range(300):
        rnd = random.Random(seed)
        T = rnd.choice([8, 16])
        if not simulate(3, T, rnd.randrange(0, 3 * T), rnd.randrange(T, 10 * T), seed,
                        drop_rule=rule):
            failures += 1
    assert failures > 0
