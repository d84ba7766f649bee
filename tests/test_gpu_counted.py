"""The counted single fill against the oracle, bit for bit.

One kernel counts the accepted pairs of every 512-pair chunk of the stream
(chunk 0 starts at the stream position, the others on the 512-pair grid),
a two-level scan (4096 chunks per workgroup, then one workgroup over the
block totals) turns the counts into exact offsets, and a second kernel
produces every chunk at its offset: 16-byte stores where a chunk has no
rejection, ranks otherwise; the last chunk continues until n outputs.
Cases:

* every word width from 2 to 32 in steps, start positions anywhere in a
  chunk, sizes around a window, a chunk and a scan block, ragged tails;
* fills spanning many scan blocks (the top level) at high rejection rates;
* misaligned outputs (the 16-byte stores shift);
* consecutive fills of one stream (positions and parity carry over);
* the test generator, the maps of Eq. (4) and 1 - z;
* no planned slack (the last chunk takes every rejection);
* generators without the form (they take another path).
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import note

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAN_BITS = np.uint64(0x7FF8DEADBEEF0001)
OGEN = {"philox": O.GEN_PHILOX, "enumerate": O.GEN_ENUMERATE, "mixed": O.GEN_MIXED,
        "mrg32k3a": O.GEN_MRG32K3A}
OMAP = {"eq5": O.MAP_EQ5, "eq4": O.MAP_EQ4, "one_minus": O.MAP_ONE_MINUS}


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for gen, w in [("philox", w) for w in range(2, 33)] + [("enumerate", w) for w in range(2, 17)] \
            + [("mrg32k3a", 32), ("mixed", 32)]:
        prngd.reset_tuning(gen, w)


def assert_bits_equal(got, expect, what):
    g = np.ascontiguousarray(got).view(np.uint64)
    e = np.ascontiguousarray(expect).view(np.uint64)
    if not np.array_equal(g, e):
        bad = np.flatnonzero(g != e)
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {i}: "
                             f"{got[i]!r} vs {expect[i]!r}")


def counted(gen, w, seed, counter, sizes, map="eq5", misalign=False, slack_mode=0,
            stream_id=0):
    """Consecutive counted fills of one stream, one per size, each compared
    in full with the guard words around it."""
    prngd.set_tuning(gen, w, path="counted", slack_mode=slack_mode)
    g = prngd.Generator(seed, gen, w=w, map=map)
    g.set_position(stream_id, counter)
    ref = O.PRNGD(OGEN[gen], w, seed=seed, stream=stream_id, counter=counter, map=OMAP[map])
    off = 1 if misalign else 2
    for i, n in enumerate(sizes):
        note(f"counted {gen} w={w} map={map} seed={seed} fill {i}: n={n} from "
             f"{ref.counter} misalign={misalign} slack={slack_mode}")
        buf = torch.empty(n + 4, dtype=torch.float64, device=DEV)
        buf.view(torch.int64).fill_(int(NAN_BITS))
        g.fill(buf[off:off + n])
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        bits = host.view(np.uint64)
        assert np.all(bits[:off] == NAN_BITS) and np.all(bits[off + n:] == NAN_BITS), \
            f"fill {i}: guard overwritten"
        expect = ref.fill(n)
        assert_bits_equal(host[off:off + n], expect, f"{gen} w={w} fill {i} n={n}")
        assert g.get_position() == (stream_id, ref.counter), f"fill {i}: position"
    g.close()


@pytest.mark.parametrize("w", [2, 3, 5, 8, 12, 16, 17, 20, 24, 27, 32])
def test_word_widths_and_start_positions(w):
    for seed, counter in [(1, 0), (2, 7), (3, 511), (4, 512), (5, 513), (6, 2**33 - 1)]:
        counted("philox", w, seed, counter, [1, 100003])


@pytest.mark.parametrize("w", [3, 24, 32])
@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 255, 256, 511, 512, 513, 1023, 1024, 4097])
def test_sizes_around_windows_and_chunks(w, n):
    counted("philox", w, 40 + n, 300, [n, n, n])


@pytest.mark.parametrize("w", [2, 3, 24])
def test_fills_spanning_many_scan_blocks(w):
    # 4096 chunks of 512 pairs per scan block: 2^23 outputs at w = 2 take
    # about 24 blocks, at w = 24 about 4; the second fill starts mid-chunk
    counted("philox", w, 77, 5, [(1 << 23) + 333, 3 * (1 << 21) + 1])


@pytest.mark.parametrize("w", [3, 24, 32])
def test_misaligned_output(w):
    counted("philox", w, 9, 129, [1, 129, 100003, 1 << 20], misalign=True)


@pytest.mark.parametrize("w", [3, 24])
def test_without_planned_slack(w):
    counted("philox", w, 11, 64, [1000, 100003, 1 << 20], slack_mode=1)


@pytest.mark.parametrize("w,n", [(4, 224), (6, 3000), (8, 254 * 256), (12, 5_000_000)])
def test_the_test_generator(w, n):
    counted("enumerate", w, 0, 0, [n, 1000])


@pytest.mark.parametrize("map", ["eq4", "one_minus"])
@pytest.mark.parametrize("w", [8, 32])
def test_map_variants(map, w):
    counted("philox", w, 13, 1001, [100003, 1 << 18], map=map)


def test_substreams():
    counted("philox", 20, 5, 0, [300001], stream_id=3)
    counted("philox", 20, 5, 12345, [300001], stream_id=2**32 - 1)


@pytest.mark.parametrize("gen", ["mixed", "mrg32k3a"])
def test_generators_without_the_form(gen):
    counted(gen, 32, 21, 17, [100003, 1 << 19])
