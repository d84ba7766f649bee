"""Every launch shape the autotuner can choose, against the oracle.

The autotuner (``autotune.candidates``) times threads per workgroup (256,
512, 1024), pairs per lane (2 to 32), store width (16-byte or
nontemporal), the ordered or speculative path and how many tiles a request
may have and still be produced by one workgroup -- and whichever is
fastest on the box becomes the launch of the resident batch.  Tuning must
never change a byte, so each candidate runs here, exactly as the batch
would run it, on:

* an uneven batch of 200 requests (sizes 1 .. 3e4, random seeds, substreams
  and start positions, odd and mid-block starts included) with
  prngd_fill_batch;
* a resident plan over the same handles, replayed twice;
* one long single fill from an odd start position;

at w = 3 and w = 8 (rejections in most windows: ranks, scans, look-back
and repair all run) and at w = 32 (the rare-rejection form the benchmark
times), plus the MRG32k3a and mixed generators' candidates.  Outputs and
final positions must equal the oracle's bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import oracle_parallel as OP
from gpu_util import DEV, Arena, assert_device_bits_equal, note, upload

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import autotune, prngd, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

OGEN = {"philox": O.GEN_PHILOX, "mrg32k3a": O.GEN_MRG32K3A, "mixed": O.GEN_MIXED}


def shape_id(c):
    keys = [("block_threads", "t"), ("pairs_per_lane", "ppl"), ("store_mode", "st"),
            ("path", "path"), ("seq_max_tiles", "seq")]
    return "-".join(f"{short}{c[k]}" for k, short in keys if k in c)


PHILOX_SHAPES = autotune.candidates("philox", 32)
MRG_SHAPES = autotune.candidates("mrg32k3a", 32)
assert autotune.candidates("mixed", 32) == MRG_SHAPES


class Expected:
    """The oracle's outputs for the test sequence of one (generator, w):
    three consecutive launches of the batch, then the single fill."""

    def __init__(self, gen, w):
        self.gen, self.w = gen, w
        self.reqs = workloads.uneven_batch(count=200, lo=1, hi=3e4, rng_seed=1000 + w)
        specs = [(r.seed, r.stream_id, r.counter, r.n) for r in self.reqs]
        self.launches = []
        for _ in range(3):
            outs, ctrs = OP.fill_streams(OGEN[gen], w, specs)
            self.launches.append((upload(outs), ctrs))
            specs = [(s[0], s[1], c, s[3]) for s, c in zip(specs, ctrs)]
        self.single_n = (1 << 20) + 3 if w == 32 else 300001
        self.single_counter = 2**33 + 12345
        s = O.PRNGD(OGEN[gen], w, seed=77, stream=5, counter=self.single_counter)
        self.single = upload([s.fill(self.single_n)])
        self.single_end = s.counter


_cache = {}


@pytest.fixture(scope="module", autouse=True)
def _release_expected():
    yield
    _cache.clear()
    torch.cuda.empty_cache()


def expected(gen, w):
    if (gen, w) not in _cache:
        _cache[(gen, w)] = Expected(gen, w)     # tens of MB on the device each
    return _cache[(gen, w)]


def run_shape(gen, w, shape):
    ex = expected(gen, w)
    prngd.set_tuning(gen, w, **shape)
    try:
        reqs = ex.reqs
        gens = []
        for r in reqs:
            g = prngd.Generator(r.seed, gen, w=w)
            g.set_position(r.stream_id, r.counter)
            gens.append(g)
        arena = Arena([r.n for r in reqs])
        arena.poison()
        note(f"shape {shape_id(shape)} {gen} w={w}: fill_batch")
        prngd.fill_batch(list(zip(gens, arena.views)))
        torch.cuda.synchronize()
        dev, ctrs = ex.launches[0]
        assert_device_bits_equal(arena.data, dev, "fill_batch", arena.offsets)
        for i, g in enumerate(gens):
            assert g.get_position() == (reqs[i].stream_id, ctrs[i]), f"fill_batch request {i}"
        plan = prngd.Plan(list(zip(gens, arena.views)))
        for rep in (1, 2):
            note(f"shape {shape_id(shape)} {gen} w={w}: plan replay {rep}")
            arena.poison()
            plan.launch()
            torch.cuda.synchronize()
            dev, ctrs = ex.launches[rep]
            assert_device_bits_equal(arena.data, dev, f"plan replay {rep}", arena.offsets)
            for i, g in enumerate(gens):
                assert g.get_position() == (reqs[i].stream_id, ctrs[i]), \
                    f"replay {rep} request {i}"
        plan.close()
        for g in gens:
            g.close()
        note(f"shape {shape_id(shape)} {gen} w={w}: single fill of {ex.single_n}")
        g = prngd.Generator(77, gen, w=w)
        g.set_position(5, ex.single_counter)
        out = Arena([ex.single_n])
        out.poison()
        g.fill(out.views[0])
        torch.cuda.synchronize()
        assert_device_bits_equal(out.data, ex.single, "single fill")
        assert g.get_position() == (5, ex.single_end)
        g.close()
    finally:
        prngd.reset_tuning(gen, w)


@pytest.mark.parametrize("w", [3, 8, 32])
@pytest.mark.parametrize("shape", PHILOX_SHAPES, ids=[shape_id(c) for c in PHILOX_SHAPES])
def test_philox_launch_shape(shape, w):
    run_shape("philox", w, shape)


@pytest.mark.parametrize("gen", ["mrg32k3a", "mixed"])
@pytest.mark.parametrize("shape", MRG_SHAPES, ids=[shape_id(c) for c in MRG_SHAPES])
def test_mrg_launch_shape(shape, gen):
    run_shape(gen, 32, shape)


def test_the_shape_the_benchmark_chose():
    # the resident batch of the uneven-batch benchmark ran in this shape
    shape = {"block_threads": 256, "pairs_per_lane": 32, "store_mode": 2, "path": 2}
    assert shape in PHILOX_SHAPES
    for w in (32, 8):
        run_shape("philox", w, shape)
