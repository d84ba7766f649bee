"""The chunk-speculative batch form against the oracle, bit for bit.

Every chunk (1, 2 or 4 windows of 128 pairs) of every request stores at
the offset it would have
if no earlier chunk of its request rejected a pair; a request with a
rejection is produced again from its first such chunk by the repair
kernel.  Cases:

* uneven batches (sizes 1 .. 3e4, random seeds, substreams and start
  positions) at w = 2, 3 (most chunks reject), 8, 12, 24, 32 and the test
  generator, by prngd_fill_batch and as a plan replayed three times;
* every chunk size (1, 2 or 4 windows of 128 pairs);
* batches of equal requests (the chunk -> request map is a division by a
  multiply-high), from start positions anywhere in a chunk, at sizes
  around a window and a chunk;
* no planned slack (the last planned chunk of a request continues until
  its n outputs, through many rejections at w = 3);
* the maps of Eq. (4) and 1 - z;
* guard words after the last request, empty requests in the batch, and
  generators without the form (they take another speculative form).
"""
import numpy as np
import pytest

import oracle as O
import oracle_parallel as OP
from gpu_util import NAN_BITS, Arena, assert_device_bits_equal, note, upload

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

OGEN = {"philox": O.GEN_PHILOX, "enumerate": O.GEN_ENUMERATE, "mixed": O.GEN_MIXED,
        "mrg32k3a": O.GEN_MRG32K3A}
OMAP = {"eq5": O.MAP_EQ5, "eq4": O.MAP_EQ4, "one_minus": O.MAP_ONE_MINUS}


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for gen, w in [("philox", w) for w in range(2, 33)] + [("enumerate", w) for w in range(2, 17)] \
            + [("mrg32k3a", 32), ("mixed", 32)]:
        prngd.reset_tuning(gen, w)


def handles(specs, gen, w, map="eq5"):
    gens = []
    for seed, stream, counter, _ in specs:
        g = prngd.Generator(seed, gen, w=w, map=map)
        g.set_position(stream, counter)
        gens.append(g)
    return gens


def run_batch(gen, w, specs, launches=4, map="eq5", slack_mode=0, ppl=0):
    """prngd_fill_batch once, then a plan replayed launches - 1 times, each
    launch compared in full (outputs, the guard after them, positions)."""
    prngd.set_tuning(gen, w, path="speculative-chunk", slack_mode=slack_mode, pairs_per_lane=ppl)
    gens = handles(specs, gen, w, map)
    arena = Arena([s[3] for s in specs] + [64])        # the last view is a guard
    views = arena.views[:-1]
    plan = None
    for launch in range(launches):
        note(f"chunk form {gen} w={w} map={map} slack={slack_mode} ppl={ppl} "
             f"{len(specs)} requests launch {launch}")
        arena.poison()
        if launch == 0:
            prngd.fill_batch(list(zip(gens, views)))
        else:
            if plan is None:
                plan = prngd.Plan(list(zip(gens, views)))
            plan.launch()
        torch.cuda.synchronize()
        outs, ctrs = OP.fill_streams(OGEN[gen], w, specs, map=OMAP[map])
        total = int(arena.offsets[-2])
        assert_device_bits_equal(arena.buf[:total], upload(outs, total), f"launch {launch}",
                                 arena.offsets[:-1])
        guard = arena.views[-1].view(torch.int64).cpu().numpy()
        assert np.all(guard == NAN_BITS), f"launch {launch}: written past the last request"
        for i, g in enumerate(gens):
            assert g.get_position() == (specs[i][1], ctrs[i]), f"launch {launch} request {i}"
        specs = [(s[0], s[1], c, s[3]) for s, c in zip(specs, ctrs)]
    if plan is not None:
        plan.close()
    for g in gens:
        g.close()


def uneven_specs(count, hi, rng_seed):
    reqs = workloads.uneven_batch(count=count, lo=1, hi=hi, rng_seed=rng_seed)
    return [(r.seed, r.stream_id, r.counter, r.n) for r in reqs]


@pytest.mark.parametrize("gen,w", [("philox", 2), ("philox", 3), ("philox", 8), ("philox", 12),
                                   ("philox", 24), ("philox", 32), ("enumerate", 6)])
def test_uneven_batches_and_plans(gen, w):
    run_batch(gen, w, uneven_specs(200, 3e4, 500 + w))


@pytest.mark.parametrize("ppl", [2, 4, 8])
@pytest.mark.parametrize("w", [3, 32])
def test_windows_per_chunk(w, ppl):
    # chunks of ppl / 2 windows of 128 pairs
    run_batch("philox", w, uneven_specs(150, 5e3, 600 + w), launches=3, ppl=ppl)


@pytest.mark.parametrize("ppl", [2, 8])
@pytest.mark.parametrize("w", [3, 32])
@pytest.mark.parametrize("n", [1, 127, 128, 129, 511, 512, 513, 1023, 1024, 4096, 16384])
def test_equal_requests(w, n, ppl):
    rnd = np.random.default_rng(n + w)
    count = 300
    # starts anywhere in a 512-pair chunk, and on its edges and windows
    counters = [int(c) for c in rnd.integers(0, 1 << 40, count)]
    counters[:8] = [0, 127, 128, 511, 512, 513, 384, 2**33 - 1]
    specs = [(7, s, counters[s], n) for s in range(count)]
    run_batch("philox", w, specs, launches=3, ppl=ppl)


@pytest.mark.parametrize("w", [3, 8, 32])
def test_without_planned_slack(w):
    run_batch("philox", w, uneven_specs(120, 2e4, 700 + w), launches=3, slack_mode=1)


@pytest.mark.parametrize("map", ["eq4", "one_minus"])
@pytest.mark.parametrize("w", [8, 32])
def test_map_variants(map, w):
    run_batch("philox", w, uneven_specs(80, 2e4, 800 + w), launches=2, map=map)


def test_empty_requests_and_one_request():
    prngd.set_tuning("philox", 8, path="speculative-chunk")
    a = prngd.Generator(1, "philox", w=8)
    b = prngd.Generator(2, "philox", w=8)
    c = prngd.Generator(3, "philox", w=8)
    ta = torch.empty(1000, dtype=torch.float64, device="cuda:0")
    tb = torch.empty(5000, dtype=torch.float64, device="cuda:0")
    tc = torch.empty(3, dtype=torch.float64, device="cuda:0")
    note("chunk form: a batch with an empty request")
    prngd.fill_batch([(a, ta, 0), (b, tb), (c, tc)])
    torch.cuda.synchronize()
    assert a.get_position() == (0, 0)
    for g, t, seed in ((b, tb, 2), (c, tc, 3)):
        s = O.PRNGD(O.GEN_PHILOX, 8, seed=seed)
        expect = s.fill(t.numel())
        assert np.array_equal(t.cpu().numpy().view(np.uint64), expect.view(np.uint64))
        assert g.get_position() == (0, s.counter)
    note("chunk form: a batch of one request")
    prngd.fill_batch([(a, ta)])
    torch.cuda.synchronize()
    s = O.PRNGD(O.GEN_PHILOX, 8, seed=1)
    assert np.array_equal(ta.cpu().numpy().view(np.uint64), s.fill(1000).view(np.uint64))
    for g in (a, b, c):
        g.close()


@pytest.mark.parametrize("gen", ["mixed", "mrg32k3a"])
def test_generators_without_the_form(gen):
    # MRG32k3a-based streams have no chunk kernel: the path falls back
    run_batch(gen, 32, uneven_specs(60, 2e4, 900), launches=2)
