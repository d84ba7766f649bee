"""PRNGD on RANMAR words on the GPU against the oracle, bit for bit.

RANMAR (a lagged generator with 24-bit words, one of those Section 2 names)
keeps its 97 lagged values and arithmetic part per handle on the device.  A
fill up to one segment (1024 pairs) is one wave; a longer one counts every
segment's accepted pairs, scans, and produces every segment from its start
window, reached by the jump table (segments of 1024 pairs up to 4096 of
them, of 8192 pairs beyond); the last segment runs on until n outputs.  A batch gives each short request one wave and fills long ones in
segments.  Cases:

* sizes around a window (128 pairs), a segment and several segments, ragged
  tails, from several positions of several streams and seeds;
* consecutive fills of one handle (the counter and the 97-value window carry
  over), and fills after prngd_set_position;
* misaligned outputs and guard words;
* the maps of Eq. (4) and 1 - z;
* batches mixing one-wave requests and segmented ones, twice in a row, and
  handles made by prngd_create_many;
* a resident plan replayed three times, and fills after it;
* the refusals (plans of long requests, the allocation-free fill, one-word
  consumption, three words per output).
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import note

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAN_BITS = np.uint64(0x7FF8DEADBEEF0001)
OMAP = {"eq5": O.MAP_EQ5, "eq4": O.MAP_EQ4, "one_minus": O.MAP_ONE_MINUS}


def assert_bits_equal(got, expect, what):
    g = np.ascontiguousarray(got).view(np.uint64)
    e = np.ascontiguousarray(expect).view(np.uint64)
    if not np.array_equal(g, e):
        bad = np.flatnonzero(g != e)
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {i}: "
                             f"{got[i]!r} vs {expect[i]!r}")


def fills(seed, stream, counter, sizes, map="eq5", misalign=False):
    """Consecutive fills of one RANMAR handle, each compared in full with
    guard words around it, and the position after each."""
    g = prngd.Generator(seed, "ranmar", w=24, map=map)
    if stream or counter:
        g.set_position(stream, counter)
    ref = O.PRNGD(O.GEN_RANMAR, 24, seed=seed, stream=stream, counter=counter, map=OMAP[map])
    off = 1 if misalign else 2
    for i, n in enumerate(sizes):
        note(f"ranmar seed={seed} stream={stream} map={map} fill {i}: n={n} from pair "
             f"{ref.counter} misalign={misalign}")
        buf = torch.empty(n + 4, dtype=torch.float64, device=DEV)
        buf.view(torch.int64).fill_(int(NAN_BITS))
        g.fill(buf[off:off + n])
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        bits = host.view(np.uint64)
        assert np.all(bits[:off] == NAN_BITS) and np.all(bits[off + n:] == NAN_BITS), \
            f"fill {i}: guard overwritten"
        assert_bits_equal(host[off:off + n], ref.fill(n), f"fill {i} n={n}")
        assert g.get_position() == (stream, ref.counter), f"fill {i}: position"
    g.close()


@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 255, 256, 1000, 1023, 1024, 1025])
def test_one_wave_sizes(n):
    fills(1, 0, 0, [n, n, 3])


@pytest.mark.parametrize("n", [2047, 2048, 2049, 8200, 16385, 100003, 1 << 20, 4_194_000,
                               5_000_001])
def test_segmented_sizes(n):
    # fine segments up to about 2^22 pairs, coarse ones past that
    fills(2, 3, 5, [n, 1000, n])


@pytest.mark.parametrize("seed,stream,counter", [(0, 0, 0), (7, 1, 1), (9, 2**32 - 1, 12345),
                                                 (2**40 + 3, 77, 2**33 + 7), (5, 11, 2**62 + 1)])
def test_positions_and_streams(seed, stream, counter):
    fills(seed, stream, counter, [100003, 7, 20000])


def test_many_consecutive_fills():
    rnd = np.random.default_rng(3)
    fills(4, 9, 0, [int(x) for x in rnd.integers(1, 40000, 24)])


@pytest.mark.parametrize("n", [1, 129, 100003])
def test_misaligned_output(n):
    fills(6, 2, 17, [n, n], misalign=True)


@pytest.mark.parametrize("map", ["eq4", "one_minus"])
def test_map_variants(map):
    fills(8, 1, 3, [5000, 100003], map=map)


def test_set_position_moves_the_window():
    g = prngd.Generator(12, "ranmar", w=24)
    out = torch.empty(5000, dtype=torch.float64, device=DEV)
    for stream, counter in [(0, 10**6), (3, 0), (3, 12345), (0, 10**6)]:
        note(f"ranmar set_position {stream} {counter}")
        g.set_position(stream, counter)
        g.fill(out)
        torch.cuda.synchronize()
        ref = O.PRNGD(O.GEN_RANMAR, 24, seed=12, stream=stream, counter=counter)
        assert_bits_equal(out.cpu().numpy(), ref.fill(5000), f"stream {stream} from {counter}")
        assert g.get_position() == (stream, ref.counter)
    g.close()


def test_batches_of_short_and_long_requests():
    reqs = workloads.uneven_batch(count=60, lo=1, hi=2e5, rng_seed=11)
    note(f"ranmar batch of {len(reqs)} requests")
    gens, refs = [], []
    for r in reqs:
        g = prngd.Generator(r.seed, "ranmar", w=24)
        g.set_position(r.stream_id, r.counter)
        gens.append(g)
        refs.append(O.PRNGD(O.GEN_RANMAR, 24, seed=r.seed, stream=r.stream_id, counter=r.counter))
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    for rep in range(2):
        note(f"ranmar batch fill {rep}")
        prngd.fill_batch(list(zip(gens, outs)))
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"batch {rep} request {i}")
            assert gens[i].get_position() == (r.stream_id, refs[i].counter), f"request {i}"
    for g in gens:
        g.close()


def test_create_many_streams():
    note("ranmar create_many")
    gens = prngd.Generator.many(21, 300, generator="ranmar", w=24, first_stream_id=1000)
    outs = [torch.empty(777, dtype=torch.float64, device=DEV) for _ in gens]
    prngd.fill_batch(list(zip(gens, outs)))
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        ref = O.PRNGD(O.GEN_RANMAR, 24, seed=21, stream=1000 + i)
        assert_bits_equal(o.cpu().numpy(), ref.fill(777), f"stream {1000 + i}")
    for g in gens:
        g.close()


def test_resident_plans():
    reqs = workloads.uneven_batch(count=50, lo=1, hi=3e4, rng_seed=17)
    gens, refs = [], []
    for r in reqs:
        g = prngd.Generator(r.seed, "ranmar", w=24)
        g.set_position(r.stream_id, r.counter)
        gens.append(g)
        refs.append(O.PRNGD(O.GEN_RANMAR, 24, seed=r.seed, stream=r.stream_id, counter=r.counter))
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    plan = prngd.Plan(list(zip(gens, outs)))
    for rep in range(3):
        note(f"ranmar plan replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"replay {rep} request {i}")
            assert gens[i].get_position() == (r.stream_id, refs[i].counter), f"request {i}"
    plan.close()
    # the handles go on from where the plan left them
    note("ranmar fills after the plan")
    gens[0].fill(outs[0])
    torch.cuda.synchronize()
    assert_bits_equal(outs[0].cpu().numpy(), refs[0].fill(reqs[0].n), "after the plan")
    for g in gens:
        g.close()


def test_refusals():
    g = prngd.Generator(1, "ranmar", w=24)
    out = torch.empty(10, dtype=torch.float64, device=DEV)
    big = torch.empty(40000, dtype=torch.float64, device=DEV)
    with pytest.raises(prngd.PrngdError):
        prngd.Plan([(g, big)])                 # plans take requests of one wave
    with pytest.raises(prngd.PrngdError):
        g.fill_noalloc(out)
    with pytest.raises(prngd.PrngdError):
        g.set_consume("single")
    with pytest.raises(prngd.PrngdError):
        g.set_arity(3)
    g.close()
