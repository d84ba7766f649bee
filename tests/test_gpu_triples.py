"""Three words per output on the GPU against the oracle, bit for bit.

The two-word method applied twice (the paper's Conclusion): triple t is
words 3t .. 3t + 2, kept iff x1 and x2 are not a0 or a, mapped by Eq. (5)
with k' = k^3.  Cases:

* single fills at w = 3, 5, 8 (rejections in most windows: ranks, scans,
  look-back), 12, 17 (3w = 51 bits, every N3 exact in FP64), 21, 24, 26
  (the last width whose inner part is exact), 27 and 32 (the 96-bit
  rounding of N3), from counters of several residues, ragged sizes over
  several windows;
* every triple of the test generator at w = 4 (the whole grid, each value
  once);
* single fills of at least 16384 triples in the counted form (and, for
  comparison, in the ordered look-back), consecutive, from starts anywhere
  in a 4096-triple window;
* an uneven batch, its plan replayed twice, and consecutive fills;
* 2^28 outputs at w = 24 and w = 17, every output and the final position;
* the refusals of other generators, maps and consumption.
"""
import numpy as np
import pytest

import oracle as O
import oracle_parallel as OP
from gpu_util import DEV, NAN_BITS, Arena, assert_device_bits_equal, note, upload

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("w", [3, 5, 8, 12, 17, 21, 24, 26, 27, 32])
@pytest.mark.parametrize("counter,n", [(0, 1), (0, 4096), (1, 4097), (4099, 70001),
                                       (2**33 + 7, 200003)])
def test_single_fill(w, counter, n):
    note(f"triples w={w} counter={counter} n={n}")
    g = prngd.Generator(21, "philox", w=w, words=3)
    g.set_position(9, counter)
    out = Arena([n])
    out.poison()
    g.fill(out.views[0])
    torch.cuda.synchronize()
    ref = O.PRNGD(O.GEN_PHILOX, w, seed=21, stream=9, counter=counter, arity=3)
    assert_device_bits_equal(out.data, upload([ref.fill(n)]), f"w={w}")
    assert g.get_position() == (9, ref.counter)
    g.close()


@pytest.mark.parametrize("path", ["auto", "ordered"])
@pytest.mark.parametrize("gen,w", [("philox", 3), ("philox", 8), ("philox", 17), ("philox", 24),
                                   ("philox", 32), ("enumerate", 6)])
def test_long_single_fills_counted_and_ordered(gen, w, path):
    """Single fills of at least 16384 triples take the counted form (count
    every 4096-triple window, scan, produce each at its offset; the last
    window continues); path 1 keeps the ordered look-back.  Consecutive
    fills from starts anywhere in a window, sizes around windows."""
    ogen = {"philox": O.GEN_PHILOX, "enumerate": O.GEN_ENUMERATE}[gen]
    for counter, sizes in [(0, [16384, 16385, 4096 * 5 + 3]), (4095, [100003, 20000]),
                           (2**33 + 7, [1 << 20, 16384])]:
        if gen == "enumerate" and counter > 2**30:
            continue
        prngd.set_tuning(gen, w, path=path)
        g = prngd.Generator(33, gen, w=w, words=3)
        g.set_position(4, counter)
        ref = O.PRNGD(ogen, w, seed=33, stream=4, counter=counter, arity=3)
        for i, n in enumerate(sizes):
            note(f"triples {path} {gen} w={w} from {ref.counter} n={n}")
            out = Arena([n + 2])
            out.poison()
            g.fill(out.views[0][:n])
            torch.cuda.synchronize()
            expect = ref.fill(n)
            got = out.views[0].cpu().numpy()
            assert np.array_equal(got[:n].view(np.uint64), expect.view(np.uint64)), f"fill {i}"
            assert np.all(got[n:].view(np.uint64) == np.uint64(NAN_BITS)), "guard overwritten"
            assert g.get_position() == (4, ref.counter), f"fill {i}"
        g.close()
        prngd.reset_tuning(gen, w)


def test_every_triple_of_the_test_generator():
    w = 4
    kept = 14 * 14 * 16
    g = prngd.Generator(0, "enumerate", w=w, words=3)
    out = torch.empty(kept, dtype=torch.float64, device=DEV)
    g.fill(out)
    torch.cuda.synchronize()
    ref = O.PRNGD(O.GEN_ENUMERATE, w, arity=3)
    expect = ref.fill(kept)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), expect.view(np.uint64))
    assert g.get_position()[1] == ref.counter
    assert np.all(np.diff(expect) > 0)
    g.close()


@pytest.mark.parametrize("w", [8, 24, 32])
def test_batches_plans_and_consecutive_fills(w):
    reqs = workloads.uneven_batch(count=80, lo=1, hi=6e4, rng_seed=300 + w)
    gens = []
    for r in reqs:
        g = prngd.Generator(r.seed, "philox", w=w, words=3)
        g.set_position(r.stream_id, r.counter)
        gens.append(g)
    specs = [(r.seed, r.stream_id, r.counter, r.n) for r in reqs]
    arena = Arena([r.n for r in reqs])
    for launch in range(3):
        note(f"triples batch w={w} launch {launch}")
        arena.poison()
        if launch == 0:
            prngd.fill_batch(list(zip(gens, arena.views)))
        else:
            if launch == 1:
                plan = prngd.Plan(list(zip(gens, arena.views)))
            plan.launch()
        torch.cuda.synchronize()
        outs, ctrs = OP.fill_streams(O.GEN_PHILOX, w, specs, arity=3)
        assert_device_bits_equal(arena.data, upload(outs), f"launch {launch}", arena.offsets)
        for i, g in enumerate(gens):
            assert g.get_position() == (reqs[i].stream_id, ctrs[i]), f"launch {launch} req {i}"
        specs = [(s[0], s[1], c, s[3]) for s, c in zip(specs, ctrs)]
    plan.close()
    for g in gens:
        g.close()


@pytest.mark.parametrize("w", [24, 17])
def test_full_size(w):
    n = 1 << 28
    g = prngd.Generator(42, "philox", w=w, words=3)
    out = torch.empty(n, dtype=torch.float64, device=DEV)
    counter = 0
    for f in range(2):
        note(f"triples w={w} 2^28 fill {f}")
        out.view(torch.int64).fill_(0x7FF8DEADBEEF0001)
        g.fill(out)
        torch.cuda.synchronize()
        exp, end = OP.fill_long(O.GEN_PHILOX, w, 42, 0, counter, n, arity=3)
        dev = upload([exp])
        del exp
        assert_device_bits_equal(out, dev, f"w={w} fill {f}")
        del dev
        assert g.get_position() == (0, end)
        counter = end
    g.close()
    del out
    torch.cuda.empty_cache()


def test_refusals():
    m = prngd.Generator(1, "mrg32k3a")
    with pytest.raises(prngd.PrngdError) as e:
        m.set_arity(3)
    assert e.value.status == prngd.ERR_UNSUPPORTED
    m.close()
    g = prngd.Generator(1, "philox", w=12, words=3)
    assert g.get_arity() == 3
    for bad in (lambda: g.set_map("eq4"), lambda: g.set_consume("single")):
        with pytest.raises(prngd.PrngdError) as e:
            bad()
        assert e.value.status == prngd.ERR_UNSUPPORTED
    with pytest.raises(prngd.PrngdError) as e:
        g.set_arity(4)
    assert e.value.status == prngd.ERR_INVALID_ARGUMENT
    # handles of one batch share the form
    h = prngd.Generator(1, "philox", w=12)
    a, b = torch.empty(10, dtype=torch.float64, device=DEV), torch.empty(10, dtype=torch.float64,
                                                                        device=DEV)
    with pytest.raises(prngd.PrngdError):
        prngd.fill_batch([(g, a), (h, b)])
    g.set_arity(2)
    prngd.fill_batch([(g, a), (h, b)])
    torch.cuda.synchronize()
    g.close()
    h.close()
