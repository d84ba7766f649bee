"""C-ABI checks that need no GPU: the library loads, exports every call the
header declares, validates arguments on the host, and computes the
constants of Eq. (5) exactly."""
import ctypes
import os
import re
import subprocess
from fractions import Fraction

import pytest

from paper_1401_8230_amd import prngd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prngd.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(prngd_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = prngd.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", prngd.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (prngd_\w+)", out))
    assert set(names) <= exported


def test_headers_are_plain_c():
    for h in HEADERS:
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", h],
                       check=True)


def test_binding_covers_every_declared_symbol():
    bound = {name for name, _, _ in prngd._SIGNATURES}
    assert set(declared_functions()) == bound


def test_status_strings():
    L = prngd.lib()
    for code, name in [(0, "PRNGD_OK"), (1, "PRNGD_ERR_INVALID_ARGUMENT"),
                       (4, "PRNGD_ERR_HIP"), (5, "PRNGD_ERR_DEVICE")]:
        assert L.prngd_status_string(code).decode() == name


CASES = [
    ("philox", w, 0, 2**w - 1, 0, 2**w - 1) for w in (2, 3, 8, 16, 24, 26, 27, 31, 32)
] + [
    ("enumerate", w, 0, 2**w - 1, 0, 2**w - 1) for w in (2, 8, 16)
] + [
    ("mrg32k3a", 32, 1, prngd.M1, 1, prngd.M1),
    ("mixed", 32, 0, 2**32 - 1, 1, prngd.M1),
]


@pytest.mark.parametrize("gen,w,a0,a,b0,b", CASES)
def test_describe_constants_are_exact(gen, w, a0, a, b0, b):
    d = prngd.describe(gen, 2.0**-w, a0, a)
    assert d["w"] == w and d["b0"] == b0 and d["b"] == b
    D = (a - a0 - 2) * 2**w + (b - b0)
    assert d["D"] == D
    assert d["S"] == float((1 - Fraction(1, 2**(2 * w))) / D)


@pytest.mark.parametrize("gen,k,lo,hi", [
    ("philox", 0.3, 0, 1),                        # k not a power of two
    ("philox", 2.0**-33, 0, 2**33 - 1),           # w > 32
    ("philox", 0.5, 0, 1),                        # w = 1: nothing accepted
    ("philox", 2.0**-8, 0, 256),                  # range is not the generator's
    ("philox", 2.0**-8, 1, 255),
    ("mrg32k3a", 2.0**-32, 0, 2**32 - 1),         # MRG range is [1, m1]
    ("mrg32k3a", 2.0**-24, 1, prngd.M1),          # MRG needs w = 32
    ("mixed", 2.0**-16, 0, 2**16 - 1),
    ("enumerate", 2.0**-17, 0, 2**17 - 1),
    ("philox", 0.0, 0, 1),
    ("philox", float("inf"), 0, 1),
    ("philox", -2.0**-8, 0, 255),
])
def test_invalid_configurations_rejected_on_host(gen, k, lo, hi):
    with pytest.raises(prngd.PrngdError) as e:
        prngd.describe(gen, k, lo, hi)
    assert e.value.status == prngd.ERR_INVALID_ARGUMENT
    # create validates before touching the GPU
    with pytest.raises(prngd.PrngdError) as e:
        prngd.Generator(1, gen, k=k, min=lo, max=hi)
    assert e.value.status == prngd.ERR_INVALID_ARGUMENT


def test_unknown_generator():
    with pytest.raises(prngd.PrngdError) as e:
        prngd.describe(7, 2.0**-8, 0, 255)
    assert e.value.status == prngd.ERR_UNSUPPORTED


def test_null_arguments():
    L = prngd.lib()
    assert L.prngd_create(1, 0, 2.0**-8, 0, 255, None) == prngd.ERR_INVALID_ARGUMENT
    assert L.prngd_fill(None, 10, None, None) == prngd.ERR_INVALID_ARGUMENT
    assert L.prngd_fill_noalloc(None, 10, None, None) == prngd.ERR_INVALID_ARGUMENT
    assert L.prngd_fill_batch(None, 0, None) == prngd.ERR_INVALID_ARGUMENT
    assert L.prngd_plan_create(None, 0, None) == prngd.ERR_INVALID_ARGUMENT
    assert L.prngd_plan_launch(None, None) == prngd.ERR_INVALID_ARGUMENT
    assert L.prngd_destroy(None) == prngd.OK
    assert L.prngd_plan_destroy(None) == prngd.OK
    sid = ctypes.c_uint32()
    ctr = ctypes.c_uint64()
    assert L.prngd_get_position(None, ctypes.byref(sid), ctypes.byref(ctr), None) == 1
    assert L.prngd_set_position(None, 0, 0, None) == prngd.ERR_INVALID_ARGUMENT


def test_tuning_round_trip_and_validation():
    prngd.set_tuning("philox", 13, pairs_per_lane=8, blocks_per_cu=3, store_mode=2)
    assert prngd.get_tuning("philox", 13) == {"pairs_per_lane": 8, "blocks_per_cu": 3,
                                              "store_mode": 2, "slack_mode": 0,
                                              "block_threads": 256, "seq_max_tiles": 0,
                                              "path": 0}
    prngd.reset_tuning("philox", 13)
    assert prngd.get_tuning("philox", 13)["pairs_per_lane"] == 16
    with pytest.raises(prngd.PrngdError):
        prngd.set_tuning("philox", 13, pairs_per_lane=6)
    with pytest.raises(prngd.PrngdError):
        prngd.set_tuning("mrg32k3a", 32, pairs_per_lane=32)
    with pytest.raises(prngd.PrngdError):
        prngd.set_tuning("philox", 13, store_mode=3)
    with pytest.raises(prngd.PrngdError):
        prngd.set_tuning("philox", 13, block_threads=128)
    with pytest.raises(prngd.PrngdError):
        prngd.set_tuning("mixed", 32, block_threads=512)
    prngd.set_tuning("philox", 13, block_threads=1024, pairs_per_lane=8)
    assert prngd.get_tuning("philox", 13)["block_threads"] == 1024
    prngd.set_tuning("philox", 13, path="speculative")
    assert prngd.get_tuning("philox", 13)["path"] == 2
    prngd.set_tuning("philox", 13, path="speculative-hold")
    assert prngd.get_tuning("philox", 13)["path"] == 3
    prngd.set_tuning("philox", 13, path="speculative-wave")
    assert prngd.get_tuning("philox", 13)["path"] == 4
    prngd.set_tuning("philox", 13, path="speculative-chunk")
    assert prngd.get_tuning("philox", 13)["path"] == 5
    prngd.set_tuning("philox", 13, path="counted")
    assert prngd.get_tuning("philox", 13)["path"] == 6
    with pytest.raises(prngd.PrngdError):
        prngd.set_tuning("philox", 13, path=7)
    prngd.set_tuning("mixed", 32, path="speculative")
    assert prngd.get_tuning("mixed", 32)["path"] == 2
    prngd.reset_tuning("mixed", 32)
    prngd.reset_tuning("philox", 13)


@pytest.mark.parametrize("gen,w,a0,a,b0,b", CASES)
def test_describe_map_constants_are_exact(gen, w, a0, a, b0, b):
    e4 = prngd.describe_map(gen, 2.0**-w, a0, a, "eq4")
    assert e4["n_offset"] == 2**w - (b - b0)
    D4 = (a - a0) * 2**w - (b - b0)
    assert e4["D"] == D4 and e4["S"] == float(Fraction(1, D4))
    e5 = prngd.describe_map(gen, 2.0**-w, a0, a, "eq5")
    om = prngd.describe_map(gen, 2.0**-w, a0, a, "one_minus")
    assert e5 == om == {"n_offset": 0, "D": (a - a0 - 2) * 2**w + (b - b0),
                        "S": prngd.describe(gen, 2.0**-w, a0, a)["S"]}


@pytest.mark.gpu
def test_map_selection_on_handles():
    g = prngd.Generator(1, "philox", w=32)
    assert g.get_map() == prngd.MAP_EQ5
    g.set_map("eq4")
    assert g.get_map() == prngd.MAP_EQ4
    with pytest.raises(prngd.PrngdError):
        g.set_map(7)
    h = prngd.Generator(1, "philox", w=32, map="one_minus")
    assert h.get_map() == prngd.MAP_ONE_MINUS
    with pytest.raises(prngd.PrngdError):
        prngd.describe_map("philox", 2.0**-8, 0, 255, 9)
