"""prngd_fill_noalloc, the entry point that allocates nothing, against
prngd_fill: the same outputs and the same new position, bit for bit, on
two calls in a row (the second with a smaller n), for Philox at w = 32 and
at w = 8 (rejections in most tiles: the look-back joins every tile), for
MRG32k3a and the mixed generator, and with three words per output; all are
also checked against the oracle.  Sizes beyond the fixed scratch are
refused before any launch.  (Named to run last: it shares one device
array with every other call on the GPU.)"""
import numpy as np
import pytest

import oracle as O
from gpu_util import DEV, Arena, assert_device_bits_equal, note, upload

torch = pytest.importorskip("torch")
from paper_1401_8230_amd import prngd  # noqa: E402

pytestmark = pytest.mark.gpu

OGEN = {"philox": O.GEN_PHILOX, "mrg32k3a": O.GEN_MRG32K3A, "mixed": O.GEN_MIXED}


@pytest.mark.parametrize("gen,w,sizes", [("philox", 32, (3_000_001, 1_000_003)),
                                         ("philox", 8, (700_001, 200_003)),
                                         ("mrg32k3a", 32, (1_000_001, 65_537)),
                                         ("mixed", 32, (1_000_001, 4_097))])
def test_noalloc_equals_fill(gen, w, sizes):
    seed, stream_id, start = 1234, 7, 2**33 + 5
    a = prngd.Generator(seed, gen, w=w)        # prngd_fill_noalloc
    b = prngd.Generator(seed, gen, w=w)        # prngd_fill
    ref = O.PRNGD(OGEN[gen], w, seed=seed, stream=stream_id, counter=start)
    for g in (a, b):
        g.set_position(stream_id, start)
    for call, n in enumerate(sizes):
        note(f"noalloc {gen} w={w} call {call} n={n}")
        oa, ob = Arena([n]), Arena([n])
        oa.poison()
        ob.poison()
        a.fill_noalloc(oa.views[0])
        b.fill(ob.views[0])
        torch.cuda.synchronize()
        assert_device_bits_equal(oa.data, ob.data, f"call {call}: noalloc vs fill")
        expect = upload([ref.fill(n)])
        assert_device_bits_equal(oa.data, expect, f"call {call}: noalloc vs oracle")
        assert a.get_position() == b.get_position() == (stream_id, ref.counter)
    a.close()
    b.close()


def test_noalloc_refuses_sizes_beyond_the_scratch():
    g = prngd.Generator(5, "philox", w=32)
    out = torch.empty(8, dtype=torch.float64, device=DEV)
    # 2^32 outputs need about 2^20 tiles of 4096 pairs; the library refuses
    # before it launches anything (so out may be short)
    rc = prngd.lib().prngd_fill_noalloc(g.handle, 2**32, out.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == prngd.ERR_INVALID_ARGUMENT
    # the handle did not move and still fills
    assert g.get_position() == (0, 0)
    g.fill_noalloc(out)
    torch.cuda.synchronize()
    ref = O.PRNGD(O.GEN_PHILOX, 32, seed=5).fill(8)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    g.close()


def test_noalloc_refuses_one_word_consumption():
    g = prngd.Generator(5, "philox", w=8, consume="single")
    out = torch.empty(16, dtype=torch.float64, device=DEV)
    with pytest.raises(prngd.PrngdError) as e:
        g.fill_noalloc(out)
    assert e.value.status == prngd.ERR_UNSUPPORTED
    g.close()


def test_noalloc_with_three_words():
    g = prngd.Generator(8, "philox", w=17, words=3)
    ref = O.PRNGD(O.GEN_PHILOX, 17, seed=8, arity=3)
    for n in (300001, 4097):
        note(f"noalloc three words n={n}")
        out = Arena([n])
        out.poison()
        g.fill_noalloc(out.views[0])
        torch.cuda.synchronize()
        assert_device_bits_equal(out.data, upload([ref.fill(n)]), f"noalloc n={n}")
        assert g.get_position() == (0, ref.counter)
    g.close()
