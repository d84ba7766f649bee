"""GPU parity: libprngd's HIP fills against the CPU oracle, bit for bit.

Integer state (pair counters) must match exactly and every FP64 output must
match to 0 ulp.  Sizes span several tiles and ragged tails; the high
rejection rates of small w exercise the compaction and the look-back.
"""
import sys

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd  # noqa: E402

pytestmark = pytest.mark.gpu

OGEN = {"philox": O.GEN_PHILOX, "mrg32k3a": O.GEN_MRG32K3A, "mixed": O.GEN_MIXED,
        "enumerate": O.GEN_ENUMERATE}
DEV = "cuda:0"
NAN_BITS = np.uint64(0x7FF8DEADBEEF0001)


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    for gen, w in [("philox", w) for w in range(2, 33)] + [("enumerate", w) for w in range(2, 17)] \
            + [("mrg32k3a", 32), ("mixed", 32)]:
        prngd.reset_tuning(gen, w)


def guarded(n, misalign=False):
    """An output view with guard words around it, pre-filled with a NaN
    pattern the kernels can never produce."""
    buf = torch.empty(n + 4, dtype=torch.float64, device=DEV)
    buf.view(torch.int64).fill_(int(NAN_BITS))
    off = 1 if misalign else 2
    return buf, buf[off:off + n]


def check_guards(buf, n, misalign=False):
    host = buf.cpu().numpy().view(np.uint64)
    off = 1 if misalign else 2
    assert np.all(host[:off] == NAN_BITS) and np.all(host[off + n:] == NAN_BITS), "guard overwritten"


def assert_bits_equal(got, expect, what):
    g = np.ascontiguousarray(got).view(np.uint64)
    e = np.ascontiguousarray(expect).view(np.uint64)
    if not np.array_equal(g, e):
        bad = np.flatnonzero(g != e)
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {i}: "
                             f"{got[i]!r} vs {expect[i]!r}")


def gpu_fill(gen, w, seed, stream_id, counter, n, misalign=False):
    g = prngd.Generator(seed, gen, w=w)
    if stream_id or counter:
        g.set_position(stream_id, counter)
    buf, out = guarded(n, misalign)
    g.fill(out)
    torch.cuda.synchronize()
    res = out.cpu().numpy().copy()
    check_guards(buf, n, misalign)
    pos = g.get_position()
    g.close()
    return res, pos


OMAP = {"eq5": O.MAP_EQ5, "eq4": O.MAP_EQ4, "one_minus": O.MAP_ONE_MINUS}


def oracle_fill(gen, w, seed, stream_id, counter, n, map="eq5"):
    s = O.PRNGD(OGEN[gen], w, seed=seed, stream=stream_id, counter=counter, map=OMAP[map])
    out = s.fill(n)
    return out, s.counter


def parity(gen, w, seed=42, stream_id=0, counter=0, n=10000, misalign=False):
    note(f"{gen} w={w} seed={seed} stream={stream_id} counter={counter} n={n} misalign={misalign}")
    got, (sid, ctr) = gpu_fill(gen, w, seed, stream_id, counter, n, misalign)
    expect, ectr = oracle_fill(gen, w, seed, stream_id, counter, n)
    assert_bits_equal(got, expect, f"{gen} w={w} n={n}")
    assert sid == stream_id
    assert ctr == ectr, f"counter {ctr} vs oracle {ectr}"
    return got


# ------------------------------------------------------------- single fills

def test_c1_philox_w32_2_20_outputs():
    parity("philox", 32, seed=42, n=1 << 20)


@pytest.mark.parametrize("w", [2, 3, 5, 8, 12, 16, 24, 26, 27, 31])
def test_philox_word_widths(w):
    parity("philox", w, seed=1000 + w, stream_id=w, n=100003)


def test_enumerate_w8_exhaustive():
    # all 2^16 pairs: 512 rejected, every accepted grid value once, in order
    got = parity("enumerate", 8, n=254 * 256)
    assert np.all(np.diff(got) > 0) and got[0] == 0.0


@pytest.mark.parametrize("w,n", [(2, 12), (4, 224), (6, 3000), (12, 5_000_000)])
def test_enumerate_other_widths(w, n):
    parity("enumerate", w, n=n)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 128, 129, 4095, 4096, 4097,
                               8191, 8193, 12289, 65537])
def test_sizes_around_tile_edges(n):
    parity("philox", 32, seed=7, n=n)
    parity("philox", 8, seed=7, n=n)


@pytest.mark.parametrize("counter", [1, 3, 4095, 4097, 2**33 - 5, 2**33 + 1, 2**40 + 12345,
                                     2**63 + 7, 2**64 - 2**21])
def test_start_positions(counter):
    # odd starts begin mid-Philox-block; 2^33 - 5 crosses the low-word carry
    parity("philox", 32, seed=9, counter=counter, n=20001)
    parity("philox", 8, seed=9, counter=counter, n=9001)


@pytest.mark.parametrize("stream_id", [1, 2**31, 2**32 - 1])
def test_substreams(stream_id):
    parity("philox", 32, seed=2**64 - 1, stream_id=stream_id, n=30000)


def test_misaligned_output():
    parity("philox", 32, seed=5, n=40001, misalign=True)
    parity("philox", 8, seed=5, n=40001, misalign=True)
    parity("mixed", 32, seed=5, n=20001, misalign=True)


@pytest.mark.parametrize("gen", ["mrg32k3a", "mixed"])
@pytest.mark.parametrize("seed,stream_id,counter,n", [
    (0, 0, 0, 1), (0, 0, 0, 50000), (42, 0, 0, 70001), (42, 3, 17, 33333),
    (2**64 - 1, 2**32 - 1, 2**40 + 5, 20000), (12345, 77, 2**62 + 1, 9999),
])
def test_mrg_generators(gen, seed, stream_id, counter, n):
    parity(gen, 32, seed=seed, stream_id=stream_id, counter=counter, n=n)


# ----------------------------------------------------- tails and tuning

@pytest.mark.parametrize("gen,w", [("philox", 2), ("philox", 3), ("philox", 8),
                                   ("enumerate", 4), ("mixed", 32), ("philox", 32)])
def test_tail_path_without_planned_slack(gen, w):
    # plan no rejections at all: every rejection is absorbed by the tail path
    prngd.set_tuning(gen, w, slack_mode=1)
    parity(gen, w, seed=11, counter=5, n=50001)


@pytest.mark.parametrize("ppl", [4, 8, 16, 32])
@pytest.mark.parametrize("store_mode", [0, 1, 2])
def test_launch_shapes_do_not_change_bytes(ppl, store_mode):
    prngd.set_tuning("philox", 32, pairs_per_lane=ppl, store_mode=store_mode)
    prngd.set_tuning("philox", 8, pairs_per_lane=ppl, store_mode=store_mode, blocks_per_cu=1)
    parity("philox", 32, seed=3, counter=1, n=100001)
    parity("philox", 8, seed=3, counter=1, n=100001)


@pytest.mark.parametrize("ppl", [4, 8, 16])
def test_mrg_launch_shapes(ppl):
    prngd.set_tuning("mixed", 32, pairs_per_lane=ppl)
    prngd.set_tuning("mrg32k3a", 32, pairs_per_lane=ppl, blocks_per_cu=1)
    parity("mixed", 32, seed=3, counter=3, n=30001)
    parity("mrg32k3a", 32, seed=3, counter=3, n=30001)


# ------------------------------------------------ sequences of fills

def test_split_fills_concatenate():
    rng = np.random.default_rng(1)
    for gen, w in [("philox", 32), ("philox", 8), ("mixed", 32)]:
        note(f"split {gen} w={w}")
        g = prngd.Generator(77, gen, w=w)
        parts = [int(v) for v in rng.integers(1, 30000, size=12)]
        outs = []
        for n in parts:
            t = torch.empty(n, dtype=torch.float64, device=DEV)
            g.fill(t)
            outs.append(t)
        torch.cuda.synchronize()
        got = torch.cat(outs).cpu().numpy()
        expect, ectr = oracle_fill(gen, w, 77, 0, 0, sum(parts))
        assert_bits_equal(got, expect, f"split {gen}")
        assert g.get_position()[1] == ectr
        g.close()


def test_checkpoint_resume():
    g = prngd.Generator(31, "philox", w=8)
    a = torch.empty(12345, dtype=torch.float64, device=DEV)
    g.fill(a)
    sid, ctr = g.get_position()
    g2 = prngd.Generator(31, "philox", w=8)
    g2.set_position(sid, ctr)
    b = torch.empty(5000, dtype=torch.float64, device=DEV)
    c = torch.empty(5000, dtype=torch.float64, device=DEV)
    g.fill(b)
    g2.fill(c)
    torch.cuda.synchronize()
    assert_bits_equal(b.cpu().numpy(), c.cpu().numpy(), "resume")
    assert g.get_position() == g2.get_position()


@pytest.mark.parametrize("path", ["ordered", "speculative", "speculative-hold",
                                  "speculative-wave"])
def test_repeated_high_rejection_fills(path):
    # many launches in a row: stale status words (ordered path) or rejection
    # list entries (speculative path) of earlier launches must never be
    # taken for the current one
    prngd.set_tuning("philox", 3, path=path)
    rng = np.random.default_rng(2)
    g = prngd.Generator(5, "philox", w=3)
    ref = O.PRNGD(O.GEN_PHILOX, 3, seed=5)
    for i in range(40):
        n = int(rng.integers(1, 200000))
        t = torch.empty(n, dtype=torch.float64, device=DEV)
        g.fill(t)
        expect = ref.fill(n)
        assert_bits_equal(t.cpu().numpy(), expect, f"fill {i}")
    assert g.get_position()[1] == ref.counter


def test_fill_on_another_stream_is_ordered():
    g = prngd.Generator(8, "philox", w=8)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = torch.empty(300000, dtype=torch.float64, device=DEV)
    b = torch.empty(300000, dtype=torch.float64, device=DEV)
    g.fill(a, stream=s1)
    g.fill(b, stream=s2)
    torch.cuda.synchronize()
    expect = O.PRNGD(O.GEN_PHILOX, 8, seed=8).fill(600000)
    assert_bits_equal(np.concatenate([a.cpu().numpy(), b.cpu().numpy()]), expect, "two streams")


# ------------------------------------------------------------- batches

def make_handles(reqs, gen, w):
    gens = []
    for r in reqs:
        g = prngd.Generator(r.seed, gen, w=w)
        if r.stream_id or r.counter:
            g.set_position(r.stream_id, r.counter)
        gens.append(g)
    return gens


@pytest.mark.parametrize("gen,w", [("philox", 32), ("philox", 8), ("mixed", 32), ("mrg32k3a", 32)])
@pytest.mark.parametrize("seq_max_tiles", [0, 1, 3, 1 << 20])
def test_batch_matches_oracle(gen, w, seq_max_tiles):
    """Requests split between the segment-sequential kernel and the
    look-back kernel in every proportion give the oracle's bytes."""
    from paper_1401_8230_amd import workloads
    note(f"batch {gen} w={w} seq_max_tiles={seq_max_tiles}")
    prngd.set_tuning(gen, w, seq_max_tiles=seq_max_tiles, path="ordered")
    reqs = workloads.uneven_batch(count=200, lo=1, hi=3e4, rng_seed=w)
    gens = make_handles(reqs, gen, w)
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    prngd.fill_batch(list(zip(gens, outs)))
    torch.cuda.synchronize()
    for i, (r, g, o) in enumerate(zip(reqs, gens, outs)):
        expect, ectr = oracle_fill(gen, w, r.seed, r.stream_id, r.counter, r.n)
        assert_bits_equal(o.cpu().numpy(), expect, f"request {i}")
        assert g.get_position() == (r.stream_id, ectr), f"request {i}"
    for g in gens:
        g.close()


def test_batch_with_empty_requests_and_errors():
    a = prngd.Generator(1, "philox", w=32)
    b = prngd.Generator(2, "philox", w=32)
    c = prngd.Generator(3, "philox", w=8)
    ta = torch.empty(1000, dtype=torch.float64, device=DEV)
    tb = torch.empty(10, dtype=torch.float64, device=DEV)
    prngd.fill_batch([(a, ta, 0), (b, tb)])
    torch.cuda.synchronize()
    assert a.get_position()[1] == 0
    assert_bits_equal(tb.cpu().numpy(), oracle_fill("philox", 32, 2, 0, 0, 10)[0], "b")
    with pytest.raises(prngd.PrngdError):
        prngd.fill_batch([(a, ta), (a, ta)])          # repeated handle
    with pytest.raises(prngd.PrngdError):
        prngd.fill_batch([(a, ta), (c, tb)])          # mixed configurations


@pytest.mark.parametrize("seq_max_tiles", [0, 1, 1 << 20])
def test_plan_replays_advance_handles(seq_max_tiles):
    from paper_1401_8230_amd import workloads
    prngd.set_tuning("philox", 8, seq_max_tiles=seq_max_tiles)
    reqs = workloads.uneven_batch(count=64, lo=1, hi=5e4, rng_seed=9)
    gens = make_handles(reqs, "philox", 8)
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    plan = prngd.Plan(list(zip(gens, outs)))
    refs = [O.PRNGD(O.GEN_PHILOX, 8, seed=r.seed, stream=r.stream_id, counter=r.counter)
            for r in reqs]
    for rep in range(4):
        note(f"plan replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"replay {rep} request {i}")
        assert gens[5].get_position()[1] == refs[5].counter
    with pytest.raises(prngd.PrngdError):
        gens[0].fill(outs[0])                          # bound to the plan
    plan.close()
    # after the plan, the handles continue where the plan left them
    t = torch.empty(777, dtype=torch.float64, device=DEV)
    gens[3].fill(t)
    assert_bits_equal(t.cpu().numpy(), refs[3].fill(777), "after plan")
    for g in gens:
        g.close()


# ------------------------------------------------ the speculative fill

@pytest.mark.parametrize("gen,w", [("philox", 2), ("philox", 3), ("philox", 8), ("philox", 12),
                                   ("enumerate", 6), ("philox", 32), ("mixed", 32),
                                   ("mrg32k3a", 32)])
@pytest.mark.parametrize("ppl", [4, 16])
@pytest.mark.parametrize("path", ["speculative", "speculative-hold", "speculative-wave"])
def test_speculative_fill_at_any_rejection_rate(gen, w, ppl, path):
    """Speculation forced where most windows reject pairs: most tiles store
    at a wrong offset first, and the repair pass must still leave exactly
    the oracle's bytes and counter."""
    prngd.set_tuning(gen, w, path=path, pairs_per_lane=ppl)
    for counter, n in [(0, 1), (7, 4097), (3, 100003), (4095, 300001)]:
        parity(gen, w, seed=19, counter=counter, n=n)


@pytest.mark.parametrize("w", [3, 8, 24, 32])
@pytest.mark.parametrize("ppl", [2, 4, 8])
def test_wave_form_chunk_sizes(w, ppl):
    """The wave-granular single fill in chunks of ppl / 2 windows of 128
    pairs: store-first clean chunks, exact chunks, published rejections,
    hints and the repair pass."""
    prngd.set_tuning("philox", w, path="speculative-wave", pairs_per_lane=ppl)
    for counter, n in [(0, 1), (7, 4097), (3, 100003), (4095, 300001), (511, 1 << 20)]:
        parity("philox", w, seed=31, counter=counter, n=n)


@pytest.mark.parametrize("path", ["speculative", "speculative-hold", "speculative-wave"])
def test_speculative_fill_with_a_long_rejection_list(path):
    # more dirty tiles than the repair caches in LDS
    prngd.set_tuning("philox", 3, path=path, pairs_per_lane=4)
    parity("philox", 3, seed=23, counter=11, n=1 << 22)


@pytest.mark.parametrize("gen,w,path", [("philox", 3, "speculative"), ("philox", 8, "speculative"),
                                        ("philox", 32, "speculative"), ("mixed", 32, "speculative"),
                                        ("philox", 3, "speculative-hold"),
                                        ("philox", 24, "speculative-hold")])
def test_speculative_batches_and_plans(gen, w, path):
    from paper_1401_8230_amd import workloads
    prngd.set_tuning(gen, w, path=path)
    reqs = workloads.uneven_batch(count=200, lo=1, hi=3e4, rng_seed=w + 100)
    note(f"speculative batch {gen} w={w}")
    gens = make_handles(reqs, gen, w)
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    prngd.fill_batch(list(zip(gens, outs)))
    torch.cuda.synchronize()
    refs = [O.PRNGD(OGEN[gen], w, seed=r.seed, stream=r.stream_id, counter=r.counter)
            for r in reqs]
    for i, (r, o) in enumerate(zip(reqs, outs)):
        assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"request {i}")
        assert gens[i].get_position() == (r.stream_id, refs[i].counter), f"request {i}"
    plan = prngd.Plan(list(zip(gens, outs)))
    for rep in range(3):
        note(f"speculative plan replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"replay {rep} request {i}")
    plan.close()
    for i, g in enumerate(gens):
        assert g.get_position() == (reqs[i].stream_id, refs[i].counter)
        g.close()


@pytest.mark.parametrize("w", [24, 32])
def test_ordered_path_at_rare_rejections(w):
    # the look-back and segment-sequential kernels stay correct where the
    # speculative fill is the default
    from paper_1401_8230_amd import workloads
    prngd.set_tuning("philox", w, path="ordered")
    parity("philox", w, seed=42, counter=3, n=1 << 20)
    reqs = workloads.uneven_batch(count=100, lo=1, hi=3e4, rng_seed=w)
    gens = make_handles(reqs, "philox", w)
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    prngd.fill_batch(list(zip(gens, outs)))
    torch.cuda.synchronize()
    for i, (r, g, o) in enumerate(zip(reqs, gens, outs)):
        expect, ectr = oracle_fill("philox", w, r.seed, r.stream_id, r.counter, r.n)
        assert_bits_equal(o.cpu().numpy(), expect, f"request {i}")
        assert g.get_position() == (r.stream_id, ectr), f"request {i}"
        g.close()


# Full-size configurations are compared in full in test_gpu_full_size.py.


@pytest.mark.parametrize("gen,w", [("philox", 32), ("philox", 12), ("mixed", 32)])
def test_create_many_matches_individual_substreams(gen, w):
    gens = prngd.Generator.many(99, 5, gen, w=w, first_stream_id=2**32 - 5)
    for i, g in enumerate(gens):
        t = torch.empty(3001, dtype=torch.float64, device=DEV)
        g.fill(t)
        expect, ectr = oracle_fill(gen, w, 99, 2**32 - 5 + i, 0, 3001)
        assert_bits_equal(t.cpu().numpy(), expect, f"substream {i}")
        assert g.get_position() == (2**32 - 5 + i, ectr)
        g.close()
    with pytest.raises(prngd.PrngdError):
        prngd.Generator.many(99, 6, gen, w=w, first_stream_id=2**32 - 5)


# ------------------------------------------------------------ map variants

@pytest.mark.parametrize("map", ["eq4", "one_minus"])
@pytest.mark.parametrize("gen,w", [("philox", 32), ("philox", 8), ("philox", 24), ("mixed", 32),
                                   ("mrg32k3a", 32), ("enumerate", 8)])
@pytest.mark.parametrize("path", ["ordered", "speculative-hold", "speculative-wave"])
def test_map_variants_match_oracle(map, gen, w, path):
    prngd.set_tuning(gen, w, path=path)
    for counter, n in [(0, 70001), (3, 4097)]:
        note(f"map {map} {gen} w={w} {path} counter={counter} n={n}")
        g = prngd.Generator(42, gen, w=w, map=map)
        if counter:
            g.set_position(0, counter)
        buf, out = guarded(n)
        g.fill(out)
        torch.cuda.synchronize()
        check_guards(buf, n)
        expect, ectr = oracle_fill(gen, w, 42, 0, counter, n, map=map)
        assert_bits_equal(out.cpu().numpy(), expect, f"{map} {gen} w={w}")
        assert g.get_position()[1] == ectr
        g.close()


@pytest.mark.parametrize("path", ["auto", "ordered"])
def test_map_variants_in_batches_and_plans(path):
    from paper_1401_8230_amd import workloads
    prngd.set_tuning("philox", 32, path=path)
    reqs = workloads.uneven_batch(count=40, lo=1, hi=3e4, rng_seed=5)
    for map in ("eq4", "one_minus"):
        gens = make_handles(reqs, "philox", 32)
        for g in gens:
            g.set_map(map)
        outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
        prngd.fill_batch(list(zip(gens, outs)))
        plan = prngd.Plan(list(zip(gens, outs)))
        plan.launch()
        torch.cuda.synchronize()
        plan.close()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            s = O.PRNGD(O.GEN_PHILOX, 32, seed=r.seed, stream=r.stream_id, counter=r.counter,
                        map=OMAP[map])
            s.fill(r.n)
            assert_bits_equal(o.cpu().numpy(), s.fill(r.n), f"{map} request {i}")
        # a batch mixing maps is refused
        gens[1].set_map("eq5")
        with pytest.raises(prngd.PrngdError):
            prngd.fill_batch(list(zip(gens[:2], outs[:2])))
        for g in gens:
            g.close()


# ------------------------------------ Algorithm 1's single-word consumption

def single_fill(gen, w, seed, counter, n, map="eq5", misalign=False):
    g = prngd.Generator(seed, gen, w=w, consume="single", map=map)
    if counter:
        g.set_position(0, counter)
    buf, out = guarded(n, misalign)
    g.fill(out)
    torch.cuda.synchronize()
    check_guards(buf, n, misalign)
    pos = g.get_position()[1]
    g.close()
    s = O.PRNGD(OGEN[gen], w, seed=seed, counter=counter, map=OMAP[map],
                consume=O.CONSUME_SINGLE)
    expect = s.fill(n)
    return out.cpu().numpy(), expect, pos, s.counter


@pytest.mark.parametrize("gen,w", [("philox", 3), ("philox", 8), ("philox", 12), ("philox", 16),
                                   ("philox", 24), ("philox", 32), ("enumerate", 8),
                                   ("mrg32k3a", 32)])
@pytest.mark.parametrize("counter,n", [(0, 1), (0, 2048), (0, 2049), (1, 5000), (4095, 6001),
                                       (7, 100003)])
def test_single_consumption_matches_oracle(gen, w, counter, n):
    note(f"single {gen} w={w} counter={counter} n={n}")
    got, expect, pos, ectr = single_fill(gen, w, 17, counter, n)
    assert_bits_equal(got, expect, f"single {gen} w={w}")
    assert pos == ectr


@pytest.mark.parametrize("w", [8, 32])
def test_algorithm1_form_on_the_gpu(w):
    # Algorithm 1's output: one-word consumption with Eq. (4)'s map
    got, expect, pos, ectr = single_fill("philox", w, 5, 3, 300001, map="eq4", misalign=True)
    assert_bits_equal(got, expect, f"Algorithm 1 w={w}")
    assert pos == ectr


def test_single_consumption_batches_plans_and_errors():
    from paper_1401_8230_amd import workloads
    reqs = workloads.uneven_batch(count=60, lo=1, hi=5e4, rng_seed=21)
    gens = make_handles(reqs, "philox", 8)
    for g in gens:
        g.set_consume("single")
    outs = [torch.empty(r.n, dtype=torch.float64, device=DEV) for r in reqs]
    refs = [O.PRNGD(O.GEN_PHILOX, 8, seed=r.seed, stream=r.stream_id, counter=r.counter,
                    consume=O.CONSUME_SINGLE) for r in reqs]
    prngd.fill_batch(list(zip(gens, outs)))
    torch.cuda.synchronize()
    for i, (r, o) in enumerate(zip(reqs, outs)):
        assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"request {i}")
        assert gens[i].get_position() == (r.stream_id, refs[i].counter)
    plan = prngd.Plan(list(zip(gens, outs)))
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            assert_bits_equal(o.cpu().numpy(), refs[i].fill(r.n), f"replay {rep} request {i}")
    plan.close()
    # pair and single handles do not mix in one batch
    gens[0].set_consume("pair")
    with pytest.raises(prngd.PrngdError):
        prngd.fill_batch(list(zip(gens[:2], outs[:2])))
    for g in gens:
        g.close()
    m = prngd.Generator(1, "mixed", w=32)
    with pytest.raises(prngd.PrngdError) as e:
        m.set_consume("single")
    assert e.value.status == prngd.ERR_UNSUPPORTED
    m.close()


# One-word consumption of one long request across workgroups: the speculative
# form (forced, so that small w puts hundreds of candidates into one launch)
# and the automatic choice; the repair's cached rules and, with more
# candidates than it caches (the test generator from position 0 at w = 16,
# whose x1 words are 0 for 2^16 pairs in a row), its in-order re-production.
@pytest.mark.parametrize("gen,w,n,forced", [
    ("philox", 8, 16000, True), ("philox", 12, 250001, True), ("philox", 16, 2**20 + 3, True),
    ("philox", 16, 2**20 + 3, False), ("philox", 32, 2**22 + 1, False),
    ("enumerate", 16, 2**16, False), ("enumerate", 16, 2**17 + 9, True),
    ("mrg32k3a", 32, 2**21 + 5, False)])
@pytest.mark.parametrize("counter", [0, 1, 4095, 3 * 4096 + 2, 2**40 + 7])
def test_single_consumption_across_workgroups(gen, w, n, forced, counter):
    if gen == "enumerate" and counter == 2**40 + 7:
        counter = 2**33 + 5          # inside the test generator's period
    note(f"single across workgroups {gen} w={w} n={n} forced={forced} counter={counter}")
    if forced:
        prngd.set_tuning(gen, w, path=3)
    got, expect, pos, ectr = single_fill(gen, w, 23, counter, n, misalign=counter == 1)
    assert_bits_equal(got, expect, f"single {gen} w={w} n={n} counter={counter}")
    assert pos == ectr


@pytest.mark.parametrize("w,forced", [(10, True), (32, False)])
def test_single_consumption_across_workgroups_repeated(w, forced):
    # consecutive fills of one handle continue its word position on the device
    if forced:
        prngd.set_tuning("philox", w, path=3)
    g = prngd.Generator(31, "philox", w=w, consume="single")
    ref = O.PRNGD(O.GEN_PHILOX, w, seed=31, consume=O.CONSUME_SINGLE)
    for i, n in enumerate([40000, 1, 65537, 2**16, 50001]):
        note(f"repeated single fill {i} w={w} n={n}")
        buf, out = guarded(n)
        g.fill(out)
        torch.cuda.synchronize()
        check_guards(buf, n)
        assert_bits_equal(out.cpu().numpy(), ref.fill(n), f"fill {i}")
        assert g.get_position()[1] == ref.counter
    g.close()


# The speculative Philox fills choose their window origin from the output
# array's address and the start position, so that every tile after the first
# starts on a 4 KB boundary; a window then starts on a Philox block's second
# pair whenever the two disagree in parity.  Every combination, at rejection
# rates that make the repair pass redo most tiles.
@pytest.mark.parametrize("gen,w", [("philox", 8), ("philox", 32), ("enumerate", 6)])
@pytest.mark.parametrize("path", ["speculative", "speculative-hold"])
@pytest.mark.parametrize("slot", [0, 1, 2, 255, 510, 511])
def test_window_origin_on_the_4k_grid(gen, w, path, slot):
    prngd.set_tuning(gen, w, path=path)
    base = torch.empty(70000 + 1024, dtype=torch.float64, device=DEV)
    # the view's first output sits `slot` doubles into a 4 KB block
    shift = ((-base.data_ptr()) % 4096) // 8
    for counter, n in [(0, 1000), (1, 50001), (2, 50001), (600, 65536), (2**33 + 1, 69999)]:
        note(f"window origin {gen} w={w} {path} slot={slot} counter={counter} n={n}")
        off = shift + slot
        base.view(torch.int64).fill_(int(NAN_BITS))
        out = base[off:off + n]
        g = prngd.Generator(29, gen, w=w)
        g.set_position(0, counter)
        g.fill(out)
        torch.cuda.synchronize()
        host = base.cpu().numpy().view(np.uint64)
        assert np.all(host[:off] == NAN_BITS) and np.all(host[off + n:] == NAN_BITS)
        expect, ectr = oracle_fill(gen, w, 29, 0, counter, n)
        assert_bits_equal(out.cpu().numpy(), expect, f"slot {slot} counter {counter}")
        assert g.get_position()[1] == ectr
        g.close()


# The one-word fills spread over workgroups choose their window origin the
# same way, in words, from the output array's slot a within its 4 KB block
# and the start position c0: windows that start on a Philox block's first
# or third word, starts too close to the stream's beginning for the origin,
# and MRG32k3a, whose windows stay on multiples of 4096 words.
@pytest.mark.parametrize("gen,w", [("philox", 10), ("philox", 16), ("philox", 32),
                                   ("enumerate", 12), ("mrg32k3a", 32)])
@pytest.mark.parametrize("slot", [0, 1, 2, 3, 255, 511])
def test_word_window_origin_on_the_4k_grid(gen, w, slot):
    prngd.set_tuning(gen, w, path=3)
    base = torch.empty(70000 + 1024, dtype=torch.float64, device=DEV)
    shift = ((-base.data_ptr()) % 4096) // 8
    for counter, n in [(0, 40000), (1, 50001), (2, 50001), (3, 65536), (1021, 2**15),
                       (4098, 50001), (2**33 + 1, 69999)]:
        note(f"word window origin {gen} w={w} slot={slot} counter={counter} n={n}")
        off = shift + slot
        base.view(torch.int64).fill_(int(NAN_BITS))
        out = base[off:off + n]
        g = prngd.Generator(37, gen, w=w, consume="single")
        g.set_position(0, counter)
        g.fill(out)
        torch.cuda.synchronize()
        host = base.cpu().numpy().view(np.uint64)
        assert np.all(host[:off] == NAN_BITS) and np.all(host[off + n:] == NAN_BITS)
        s = O.PRNGD(OGEN[gen], w, seed=37, counter=counter, consume=O.CONSUME_SINGLE)
        assert_bits_equal(out.cpu().numpy(), s.fill(n), f"slot {slot} counter {counter}")
        assert g.get_position()[1] == s.counter
        g.close()


def _planned_pairs(n, w):
    """The pairs the library plans for n outputs of a full-range stream:
    n plus the expected rejections plus four standard deviations."""
    rho = 2.0 / 2**w
    mean = n * rho / (1.0 - rho)
    return n + int(np.floor(mean + 4.0 * np.sqrt(mean) + 0.5))


def test_lookback_tile_past_the_last_output():
    # A fill planned for more pairs than its rejections end up needing has
    # tiles that lie wholly past output n - 1.  Such a tile of the ordered
    # look-back kernel must store nothing, clean window or not.  Pick n so
    # that the last planned tile starts past the n-th accepted pair and its
    # window has no rejection, then check the outputs and a guard of two
    # windows after them.
    w, seed, T = 14, 77, 4096
    top = 1 << 24
    ref = O.PRNGD(O.GEN_PHILOX, w, seed=seed)
    _, idx = ref.fill(top + 4 * T, with_index=True)
    idx = idx.astype(np.int64)
    chosen = None
    for n in range(top - 3000, top - 1000):
        tiles = -(-_planned_pairs(n, w) // T)
        start = (tiles - 1) * T
        before = int(np.searchsorted(idx, start))          # outputs before the tile
        inside = int(np.searchsorted(idx, start + T)) - before
        if before >= n and inside == T:
            chosen = n
            break
    assert chosen is not None, "no size puts a clean tile past the last output"
    n = chosen
    prngd.set_tuning("philox", w, path=1)
    try:
        g = prngd.Generator(seed, "philox", w=w)
        base = torch.empty(n + 2 * T, dtype=torch.float64, device=DEV)
        base.view(torch.int64).fill_(int(NAN_BITS))
        note(f"look-back tile past the last output: w={w} n={n}")
        g.fill(base[:n])
        torch.cuda.synchronize()
        host = base.cpu().numpy()
        assert np.all(host[n:].view(np.uint64) == NAN_BITS), "written past output n - 1"
        expect = O.PRNGD(O.GEN_PHILOX, w, seed=seed)
        assert_bits_equal(host[:n], expect.fill(n), "outputs")
        assert g.get_position() == (0, expect.counter)
        g.close()
    finally:
        prngd.reset_tuning("philox", w)
