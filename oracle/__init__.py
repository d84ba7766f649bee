"""CPU oracle for the PRNGD method -- TEST INFRASTRUCTURE ONLY.

A plain sequential C implementation (``prngd_oracle.c``) of what the PRNGD
fill computes, written from Demchik & Gulov, arXiv:1401.8230, Section 2 and
Algorithm 1, wrapped here with ctypes.  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this package; the product path
never does.
"""
import ctypes
import os

import numpy as np

from . import build as _build

GEN_PHILOX = 0
GEN_MRG32K3A = 1
GEN_MIXED = 2
GEN_ENUMERATE = 3
GEN_RANMAR = 4

MAP_EQ5 = 0          # Eq. (5): [0, 1)
MAP_EQ4 = 1          # Eq. (4), Algorithm 1's Z: (0, 1)
MAP_ONE_MINUS = 2    # 1 - Eq. (5): (0, 1]

CONSUME_PAIR = 0     # a rejected x1 consumes the whole pair
CONSUME_SINGLE = 1   # Algorithm 1: a rejected r1 consumes one word

M1 = 4294967087
M2 = 4294944443


class Stream(ctypes.Structure):
    _fields_ = [
        ("generator", ctypes.c_int),
        ("w", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_uint32),
        ("counter", ctypes.c_uint64),
        ("a0", ctypes.c_uint64),
        ("a", ctypes.c_uint64),
        ("b0", ctypes.c_uint64),
        ("b", ctypes.c_uint64),
        ("D", ctypes.c_uint64),
        ("S", ctypes.c_double),
        ("map", ctypes.c_int),
        ("D4", ctypes.c_uint64),
        ("S4", ctypes.c_double),
        ("consume", ctypes.c_int),
        ("mrg", ctypes.c_uint32 * 6),
        ("arity", ctypes.c_int),
        ("D3_hi", ctypes.c_uint64),
        ("D3_lo", ctypes.c_uint64),
        ("S3", ctypes.c_double),
        ("ranmar", ctypes.c_uint32 * 97),
    ]


_lib = None


def lib():
    """Load the oracle library, building it only if it is not built yet."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        sp = ctypes.POINTER(Stream)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint64, ctypes.c_uint64, u32p]
        L.orc_mrg_jump.argtypes = [u32p, u64p, ctypes.c_int]
        L.orc_mrg_outputs.argtypes = [u32p, ctypes.c_uint64, u32p]
        L.orc_mrg_matpow.argtypes = [ctypes.c_int, u64p, ctypes.c_int, u64p]
        L.orc_mrg_stream_base.argtypes = [ctypes.c_uint64, ctypes.c_uint32, u32p]
        L.orc_init.argtypes = [sp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                               ctypes.c_uint32, ctypes.c_uint64]
        L.orc_init.restype = ctypes.c_int
        L.orc_init_ranges.argtypes = [sp, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint64]
        L.orc_init_ranges.restype = ctypes.c_int
        L.orc_pair.argtypes = [sp, ctypes.c_uint64, u64p, u64p]
        L.orc_accept.argtypes = [sp, ctypes.c_uint64]
        L.orc_accept.restype = ctypes.c_int
        L.orc_map.argtypes = [sp, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_map.restype = ctypes.c_double
        L.orc_fill.argtypes = [sp, ctypes.c_uint64, dp, u64p]
        L.orc_fill_pairs.argtypes = [sp, ctypes.c_uint64, ctypes.c_uint64, dp]
        L.orc_fill_pairs.restype = ctypes.c_uint64
        L.orc_scale.argtypes = [ctypes.c_int, ctypes.c_uint64]
        L.orc_scale.restype = ctypes.c_double
        L.orc_recip.argtypes = [ctypes.c_uint64]
        L.orc_recip.restype = ctypes.c_double
        L.orc_set_map.argtypes = [sp, ctypes.c_int]
        L.orc_set_consume.argtypes = [sp, ctypes.c_int]
        L.orc_word.argtypes = [sp, ctypes.c_uint64]
        L.orc_word.restype = ctypes.c_uint64
        L.orc_set_arity.argtypes = [sp, ctypes.c_int]
        L.orc_accept3.argtypes = [sp, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_accept3.restype = ctypes.c_int
        L.orc_map3.argtypes = [sp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_map3.restype = ctypes.c_double
        L.orc_rn_u128.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_rn_u128.restype = ctypes.c_double
        L.orc_scale3.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_scale3.restype = ctypes.c_double
        L.orc_ranmar_seed.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.orc_ranmar_stream_seeds.argtypes = [ctypes.c_uint64, ctypes.c_uint32, u32p, u32p]
        L.orc_ranmar_step_to.argtypes = [u32p, ctypes.c_uint64, u32p, u32p]
        L.orc_ranmar_jump.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, u32p, u32p]
        L.orc_ranmar_words.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, u32p]
        _lib = L
    return _lib


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def _limbs(e):
    e = int(e)
    limbs = []
    while e:
        limbs.append(e & (2**64 - 1))
        e >>= 64
    limbs = limbs or [0]
    return np.array(limbs, dtype=np.uint64)


def philox4x32_10(ctr, key):
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return out


def philox_words(seed, stream, first, count):
    out = np.zeros(count, dtype=np.uint32)
    lib().orc_philox_words(seed, stream, first, count, _ptr(out, ctypes.c_uint32))
    return out


def mrg_outputs(state, count):
    """``count`` outputs starting from the six-word ``state``; returns
    (outputs, new_state)."""
    st = np.array(state, dtype=np.uint32)
    out = np.zeros(count, dtype=np.uint32)
    lib().orc_mrg_outputs(_ptr(st, ctypes.c_uint32), count,
                          _ptr(out, ctypes.c_uint32))
    return out, st


def mrg_jump(state, exponent):
    st = np.array(state, dtype=np.uint32)
    e = _limbs(exponent)
    lib().orc_mrg_jump(_ptr(st, ctypes.c_uint32), _ptr(e, ctypes.c_uint64), len(e))
    return st


def mrg_matpow(component, exponent):
    e = _limbs(exponent)
    out = np.zeros(9, dtype=np.uint64)
    lib().orc_mrg_matpow(component, _ptr(e, ctypes.c_uint64), len(e),
                         _ptr(out, ctypes.c_uint64))
    return out.reshape(3, 3)


def mrg_stream_base(seed, stream):
    out = np.zeros(6, dtype=np.uint32)
    lib().orc_mrg_stream_base(seed, stream, _ptr(out, ctypes.c_uint32))
    return out


def ranmar_seed(ij, kl):
    """RANMAR's seed values L[-96..0] (the window at word position 0)."""
    out = np.zeros(97, dtype=np.uint32)
    lib().orc_ranmar_seed(ij, kl, _ptr(out, ctypes.c_uint32))
    return out


def ranmar_stream_seeds(seed, stream):
    ij, kl = ctypes.c_uint32(), ctypes.c_uint32()
    lib().orc_ranmar_stream_seeds(seed, stream, ctypes.byref(ij), ctypes.byref(kl))
    return int(ij.value), int(kl.value)


def ranmar_step_to(window0, n):
    """The window and C at word position n, by stepping."""
    w0 = np.ascontiguousarray(window0, dtype=np.uint32)
    out = np.zeros(97, dtype=np.uint32)
    C = ctypes.c_uint32()
    lib().orc_ranmar_step_to(_ptr(w0, ctypes.c_uint32), n, _ptr(out, ctypes.c_uint32),
                             ctypes.byref(C))
    return out, int(C.value)


def ranmar_jump(window0, n):
    """The window and C at word position n (< 2^128), by the jump polynomial."""
    w0 = np.ascontiguousarray(window0, dtype=np.uint32)
    out = np.zeros(97, dtype=np.uint32)
    C = ctypes.c_uint32()
    lib().orc_ranmar_jump(_ptr(w0, ctypes.c_uint32), n & (2**64 - 1), n >> 64,
                          _ptr(out, ctypes.c_uint32), ctypes.byref(C))
    return out, int(C.value)


def ranmar_words(window0, first, count):
    w0 = np.ascontiguousarray(window0, dtype=np.uint32)
    out = np.zeros(count, dtype=np.uint32)
    lib().orc_ranmar_words(_ptr(w0, ctypes.c_uint32), first, count, _ptr(out, ctypes.c_uint32))
    return out


def scale(w, D):
    return lib().orc_scale(w, D)


def rn_u128(v):
    """The oracle's round-to-nearest-even of a non-negative integer < 2^128."""
    return lib().orc_rn_u128((v >> 64) & (2**64 - 1), v & (2**64 - 1))


def scale3(w, D):
    """The oracle's RN((2^3w - 1) / (D 2^3w)) for an integer 0 < D < 2^3w."""
    return lib().orc_scale3(w, (D >> 64) & (2**64 - 1), D & (2**64 - 1))


def recip(D):
    return lib().orc_recip(D)


class PRNGD:
    """One oracle stream (sequential, single-threaded)."""

    def __init__(self, generator, w, seed=0, stream=0, counter=0, ranges=None, map=MAP_EQ5,
                 consume=CONSUME_PAIR, arity=2):
        self.s = Stream()
        if ranges is not None:
            a0, a, b0, b = ranges
            rc = lib().orc_init_ranges(ctypes.byref(self.s), w, a0, a, b0, b)
        else:
            rc = lib().orc_init(ctypes.byref(self.s), generator, w, seed, stream,
                                counter)
        if rc != 0:
            raise ValueError("invalid oracle stream parameters")
        if lib().orc_set_map(ctypes.byref(self.s), map) != 0:
            raise ValueError("unknown map")
        if lib().orc_set_consume(ctypes.byref(self.s), consume) != 0:
            raise ValueError("unknown consumption mode, or not a single-generator stream")
        if lib().orc_set_arity(ctypes.byref(self.s), arity) != 0:
            raise ValueError("three words per output need a single-generator stream, "
                             "Eq. (5) and pair consumption")

    @property
    def counter(self):
        return int(self.s.counter)

    @counter.setter
    def counter(self, value):
        self.s.counter = value

    @property
    def D(self):
        return int(self.s.D)

    @property
    def S(self):
        return float(self.s.S)

    @property
    def D4(self):
        return int(self.s.D4)

    @property
    def S4(self):
        return float(self.s.S4)

    @property
    def D3(self):
        return (int(self.s.D3_hi) << 64) | int(self.s.D3_lo)

    @property
    def S3(self):
        return float(self.s.S3)

    def accept3(self, x1, x2):
        return bool(lib().orc_accept3(ctypes.byref(self.s), x1, x2))

    def map3(self, x1, x2, x3):
        return lib().orc_map3(ctypes.byref(self.s), x1, x2, x3)

    @property
    def ranges(self):
        return int(self.s.a0), int(self.s.a), int(self.s.b0), int(self.s.b)

    def pair(self, p):
        x1 = ctypes.c_uint64()
        x2 = ctypes.c_uint64()
        lib().orc_pair(ctypes.byref(self.s), p, ctypes.byref(x1), ctypes.byref(x2))
        return int(x1.value), int(x2.value)

    def word(self, j):
        return int(lib().orc_word(ctypes.byref(self.s), j))

    def accept(self, x1):
        return bool(lib().orc_accept(ctypes.byref(self.s), x1))

    def map(self, x1, x2):
        return lib().orc_map(ctypes.byref(self.s), x1, x2)

    def fill(self, n, with_index=False):
        out = np.empty(n, dtype=np.float64)
        idx = np.empty(n, dtype=np.uint64) if with_index else None
        lib().orc_fill(ctypes.byref(self.s), n, _ptr(out, ctypes.c_double),
                       _ptr(idx, ctypes.c_uint64) if with_index else None)
        return (out, idx) if with_index else out

    def fill_pairs(self, pair_end, max_out):
        """Outputs of the accepted pairs among [counter, pair_end), at most
        max_out of them; the counter moves to the first pair not examined."""
        out = np.empty(max_out, dtype=np.float64)
        k = lib().orc_fill_pairs(ctypes.byref(self.s), pair_end, max_out,
                                 _ptr(out, ctypes.c_double))
        return out[:k]
