"""A CPU model of where the one-word (Algorithm 1) fill's words sit.

The one-word kernels take a window of T = 4096 consecutive words of a
Philox4x32-10 stream, four to a thread-block (j, tid): 256 threads, four
blocks j per thread.  A window that starts on a Philox block's first word
holds block (wb >> 2) + j * 256 + tid in thread-block (j, tid).  One that
starts on a block's third word computes the same blocks and moves words
0 and 1 of the next block in from the next lane: by a shuffle inside a
wave, from the next wave's lane 0 (or the first wave of the next j) through
LDS at a wave's edge, and from one more block, computed by the window's
last thread, at the window's end.  Every window then holds its words in
order, q = 4 (j * 256 + tid) + l for l = 0 .. 3, and a thread flags its
words q >= lo that equal a0 or a (the candidates).  A clean window pairs
them up from its entry state: (q, q + 1) for even q from state E, or
(q - 1, q) for even q from state P, the word before a thread's first taken
from the previous thread-block (a shuffle, LDS at a wave or j edge, or the
pending word for the window's first).

The model replays that index arithmetic exactly (including a wave
shuffle's behaviour at lane 63, which returns the lane's own value) and
checks, for every thread-block of many windows:

* every slot holds the word its q names, so no word of the window is
  skipped, doubled, or taken from the wrong block;
* the candidate flags are exactly the window's candidates at q >= lo;
* a clean window's pairs are exactly the pairs the sequential walk forms.

It then replays a whole one-word fill window by window -- the window
origin chosen from the output's 4 KB slot and the start parity, a clean
window paired from its entry state, any other window walked word by word
-- over the stream whose fill once failed on the GPU in a form of these
kernels that let windows start on any word (seed 17, w = 16, first word 7,
100003 outputs: word 118711 is a0, the fourth word of its Philox block),
for slots of the output in its 4 KB block of both parities (the failing
run's slot 2 among them), and compares the result
with Algorithm 1's sequential walk over the oracle's words.
"""
import numpy as np
import pytest

import oracle as O

NW, J = 4, 4
B = 64 * NW
T = 4 * J * B            # words per window


def stream_words(seed, w, first, count):
    """Words first .. first + count - 1 of a Philox stream at width w."""
    raw = O.philox_words(seed, 0, first, count).astype(np.uint64)
    return raw >> np.uint64(32 - w)


def model_single_generate(words_at, wb, lo, a0, a):
    """The kernel's u[j][l] per thread (array [J, B, 4]) and its candidate
    flag per thread, for the window starting at word wb (even)."""
    assert wb % 2 == 0
    blk0 = wb >> 2
    tid = np.arange(B)
    u = np.zeros((J, B, 4), dtype=np.uint64)
    for j in range(J):
        blocks = blk0 + j * B + tid
        for l in range(4):
            u[j, :, l] = words_at(4 * blocks + l)
    if wb & 2:
        lane, wave = tid & 63, tid >> 6
        head = {(j, wv): (u[j, wv * 64, 0], u[j, wv * 64, 1]) for j in range(J) for wv in range(NW)}
        tb = blk0 + J * B
        tail = (words_at(np.array([4 * tb]))[0], words_at(np.array([4 * tb + 1]))[0])
        new = np.zeros_like(u)
        for j in range(J):
            # __shfl_down(v, 1, 64): lane i reads lane i + 1 of its wave; lane
            # 63 has no such lane and reads its own value
            src = np.where(lane < 63, tid + 1, tid)
            n0 = u[j, src, 0].copy()
            n1 = u[j, src, 1].copy()
            for t in np.flatnonzero(lane == 63):
                wv = t >> 6
                e = head[(j, wv + 1)] if wv + 1 < NW else head[(j + 1, 0)] if j + 1 < J else tail
                n0[t], n1[t] = e
            new[j, :, 0] = u[j, :, 2]
            new[j, :, 1] = u[j, :, 3]
            new[j, :, 2] = n0
            new[j, :, 3] = n1
        u = new
    q = 4 * (np.arange(J)[:, None, None] * B + tid[None, :, None]) + np.arange(4)[None, None, :]
    cand = (u == a0) | (u == a)
    flags = np.any(cand & (q >= lo), axis=(0, 2))
    return u, q, flags


def clean_pairs(u, wb, state, pending_word_index):
    """Word indices of a clean window's outputs 2m and 2m + 1 (m = j B +
    tid), as the kernel forms them from entry state E (0) or P (1)."""
    tid = np.arange(B)
    lane, wave = tid & 63, tid >> 6
    pairs = np.zeros((J, B, 2, 2), dtype=np.int64)
    qidx = (wb + 4 * (np.arange(J)[:, None] * B + tid[None, :]))   # word index of u[j][0]
    if state == 0:
        pairs[:, :, 0] = np.stack([qidx, qidx + 1], axis=-1)
        pairs[:, :, 1] = np.stack([qidx + 2, qidx + 3], axis=-1)
        return pairs.reshape(-1, 2)
    # the word before thread-block m's first: lane i - 1's u[3] (shfl_up);
    # lane 0 reads `last` of the previous wave, of the last wave of j - 1,
    # or the pending word
    last = {(j, wv): qidx[j, wv * 64 + 63] + 3 for j in range(J) for wv in range(NW)}
    for j in range(J):
        for t in range(B):
            if lane[t] > 0:
                prev = qidx[j, t - 1] + 3
            elif wave[t] > 0:
                prev = last[(j, wave[t] - 1)]
            elif j > 0:
                prev = last[(j - 1, NW - 1)]
            else:
                prev = pending_word_index
            pairs[j, t, 0] = (prev, qidx[j, t])
            pairs[j, t, 1] = (qidx[j, t] + 1, qidx[j, t] + 2)
    return pairs.reshape(-1, 2)


@pytest.mark.parametrize("w", [3, 16, 32])
@pytest.mark.parametrize("wb", [0, 2, 4096 * 28 + 2, 118708 - 4020 + 2, 4 * (2**32 - 512) + 2,
                                4 * (2**32 - 300), 8 * (2**40) + 6])
def test_every_slot_holds_its_word(w, wb):
    seed = 17
    a0, a = 0, (1 << w) - 1
    base = max(wb - 8, 0)
    ws = stream_words(seed, w, base, T + 16)

    def words_at(idx):
        return ws[np.asarray(idx) - base]
    for lo in (0, 1, 2, 5, 2047, 4095):
        u, q, flags = model_single_generate(words_at, wb, lo, a0, a)
        assert np.array_equal(u, words_at(wb + q)), f"wb={wb} lo={lo}"
        truth = np.zeros(B, dtype=bool)
        window = words_at(wb + np.arange(T))
        for qq in np.flatnonzero(((window == a0) | (window == a)) & (np.arange(T) >= lo)):
            truth[(qq // 4) % B] = True
        assert np.array_equal(flags, truth), f"wb={wb} lo={lo}"


def test_clean_pairs_are_the_sequential_pairs():
    wb = 4096 * 7 + 2
    for state in (0, 1):
        got = clean_pairs(None, wb, state, wb - 1)
        # sequential pairing of a candidate-free window from state E: (wb +
        # 2k, wb + 2k + 1); from state P the pending r1 is word wb - 1
        k = np.arange(T // 2)
        if state == 0:
            want = np.stack([wb + 2 * k, wb + 2 * k + 1], axis=-1)
        else:
            want = np.stack([wb + 2 * k - 1, wb + 2 * k], axis=-1)
        order = np.argsort(got[:, 1])
        assert np.array_equal(got[order], want)


def word_lo0(slot, c0):
    """The window origin of a Philox one-word fill: words of the first
    window before c0 (the output's 8-byte slot in its 4 KB block, start
    parity), as the kernel chooses it."""
    lo = (2 * slot - (c0 & 1)) & 1023
    return lo if c0 >= lo else c0 & 1


def sequential(words, base, a0, a, c0, n):
    out, q = [], c0
    while len(out) < n:
        while words[q - base] in (a0, a):
            q += 1
        out.append((q, q + 1))
        q += 2
    return np.array(out, dtype=np.int64), q


def windowed_fill(words, base, a0, a, c0, n, slot):
    """The whole fill produced window by window with complete hints: clean
    windows paired from their entry state by the kernel's layout, other
    windows (and the clipped first one) walked word by word."""
    lo0 = word_lo0(slot, c0)
    wb = c0 - lo0
    assert wb % 2 == 0
    state, pending, out = 0, None, []

    def words_at(idx):
        return words[np.asarray(idx) - base]
    first = True
    while len(out) < n:
        lo = lo0 if first else 0
        u, q, flags = model_single_generate(words_at, wb, lo, a0, a)
        if flags.any() or lo != 0:
            for qq in range(wb + lo, wb + T):
                x = words[qq - base]
                if state == 0:
                    if x in (a0, a):
                        continue
                    state, pending = 1, qq
                else:
                    out.append((pending, qq))
                    state = 0
        else:
            pairs = clean_pairs(u, wb, state, pending)
            pairs = pairs[np.argsort(pairs[:, 1])]
            out.extend(map(tuple, pairs))
            if state == 1:
                pending = wb + T - 1
        first = False
        wb += T
    out = np.array(out[:n], dtype=np.int64)
    return out, int(out[-1, 1]) + 1


def test_the_stream_that_failed_with_any_word_windows():
    seed, w, c0, n = 17, 16, 7, 100003
    a0, a = 0, (1 << w) - 1
    span = 2 * n + 4 * T
    words = stream_words(seed, w, 0, span)
    # the word the failing form took as an accepted r1
    assert words[118711] == a0 and 118711 % 4 == 3
    truth, end = sequential(words, 0, a0, a, c0, n)
    # it is a rejected r1 of the sequential walk
    assert all(p[0] != 118711 for p in truth)
    for slot in sorted(set(range(0, 512, 23)) | {1, 2, 3, 255, 510, 511}):
        got, got_end = windowed_fill(words, 0, a0, a, c0, n, slot)
        assert np.array_equal(got, truth), f"slot {slot}"
        assert got_end == end
        # the window holding word 118711 flags it
        lo0 = word_lo0(slot, c0)
        wb = c0 - lo0 + ((118711 - (c0 - lo0)) // T) * T
        _, _, flags = model_single_generate(lambda i: words[np.asarray(i)], wb, 0, a0, a)
        assert flags[((118711 - wb) // 4) % B]


@pytest.mark.parametrize("w", [3, 5, 12])
def test_windowed_fill_matches_the_walk_at_high_rejection(w):
    rng = np.random.default_rng(w)
    a0, a = 0, (1 << w) - 1
    for _ in range(3):
        c0 = int(rng.integers(0, 5000))
        n = int(rng.integers(1, 12000))
        slot = int(rng.integers(0, 512))
        words = stream_words(99, w, 0, c0 + 4 * n + 3 * T)
        truth, end = sequential(words, 0, a0, a, c0, n)
        got, got_end = windowed_fill(words, 0, a0, a, c0, n, slot)
        assert np.array_equal(got, truth) and got_end == end
