"""Python binding of libprngd (ctypes).

Argument marshalling only: every step of a fill runs in the library's HIP
kernels.  PyTorch is used for device memory (tensors) and streams.  The
library is loaded from this package directory; if it is not built, every
call raises instead of computing anything elsewhere.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprngd.so")

PHILOX4X32_10 = 0
MRG32K3A = 1
PHILOX_X1_MRG32K3A_X2 = 2
ENUMERATE = 3
RANMAR = 4

MAP_EQ5 = 0
MAP_EQ4 = 1
MAP_ONE_MINUS = 2
MAPS = {"eq5": MAP_EQ5, "eq4": MAP_EQ4, "one_minus": MAP_ONE_MINUS}

CONSUME_PAIR = 0
CONSUME_SINGLE = 1
CONSUMES = {"pair": CONSUME_PAIR, "single": CONSUME_SINGLE}

GENERATORS = {
    "philox": PHILOX4X32_10,
    "philox4x32_10": PHILOX4X32_10,
    "mrg32k3a": MRG32K3A,
    "mixed": PHILOX_X1_MRG32K3A_X2,
    "philox_x1_mrg32k3a_x2": PHILOX_X1_MRG32K3A_X2,
    "enumerate": ENUMERATE,
    "ranmar": RANMAR,
}

M1 = 4294967087

OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_UNSUPPORTED = 2
ERR_OUT_OF_MEMORY = 3
ERR_HIP = 4
ERR_DEVICE = 5


class PrngdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(message)
        self.status = status


class Request(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("n", ctypes.c_uint64), ("out", ctypes.c_void_p)]


def _request_dtype():
    import numpy as np
    return np.dtype([("h", np.uint64), ("n", np.uint64), ("out", np.uint64)])


class Tuning(ctypes.Structure):
    _fields_ = [("pairs_per_lane", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("store_mode", ctypes.c_uint32), ("slack_mode", ctypes.c_uint32),
                ("block_threads", ctypes.c_uint32), ("seq_max_tiles", ctypes.c_uint32),
                ("path", ctypes.c_uint32)]


# (name, restype, argtypes) of every exported function
_SIGNATURES = [
    ("prngd_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("prngd_last_error", ctypes.c_char_p, []),
    ("prngd_describe", ctypes.c_int,
     [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
      ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
      ctypes.POINTER(ctypes.c_double)]),
    ("prngd_create", ctypes.c_int,
     [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
      ctypes.POINTER(ctypes.c_void_p)]),
    ("prngd_create_many", ctypes.c_int,
     [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
      ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    ("prngd_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("prngd_set_position", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]),
    ("prngd_get_position", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
      ctypes.c_void_p]),
    ("prngd_fill", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    ("prngd_fill_noalloc", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    ("prngd_fill_batch", ctypes.c_int,
     [ctypes.POINTER(Request), ctypes.c_uint32, ctypes.c_void_p]),
    ("prngd_plan_create", ctypes.c_int,
     [ctypes.POINTER(Request), ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    ("prngd_plan_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("prngd_plan_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("prngd_set_tuning", ctypes.c_int,
     [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(Tuning)]),
    ("prngd_get_tuning", ctypes.c_int,
     [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(Tuning)]),
    ("prngd_describe_map", ctypes.c_int,
     [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
      ctypes.POINTER(ctypes.c_double)]),
    ("prngd_set_map", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("prngd_set_consume", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("prngd_get_consume", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    ("prngd_get_map", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    ("prngd_ranmar_state", ctypes.c_int,
     [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)]),
    ("prngd_set_arity", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    ("prngd_get_arity", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    ("prngd_probe_write", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    ("prngd_probe_copy", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    ("prngd_probe_philox", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]),
    ("prngd_probe_set_spin_limit", ctypes.c_int, [ctypes.c_uint32]),
    ("prngd_probe_philox_store", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
]

_lib = None


def lib():
    """The loaded libprngd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PrngdError(ERR_UNSUPPORTED,
                             f"{LIB_PATH} is not built: run python -m paper_1401_8230_amd._build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        L = lib()
        name = L.prngd_status_string(status).decode()
        msg = L.prngd_last_error().decode()
        raise PrngdError(status, f"{name}: {msg}")


def _gen(generator):
    if isinstance(generator, str):
        return GENERATORS[generator.lower()]
    return int(generator)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _out_ptr(out, n):
    import torch
    if not isinstance(out, torch.Tensor):
        raise TypeError("out must be a torch tensor")
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 CUDA tensor")
    if n is None:
        n = out.numel()
    if n > out.numel():
        raise ValueError(f"n = {n} exceeds the {out.numel()} elements of out")
    return out.data_ptr(), int(n)


def describe(generator, k, min, max):
    """Constants of Eq. (5) for (generator, k, min, max), host only."""
    w = ctypes.c_uint32()
    b0 = ctypes.c_uint64()
    b = ctypes.c_uint64()
    D = ctypes.c_uint64()
    S = ctypes.c_double()
    _check(lib().prngd_describe(_gen(generator), k, min, max, ctypes.byref(w),
                                ctypes.byref(b0), ctypes.byref(b), ctypes.byref(D),
                                ctypes.byref(S)))
    return {"w": w.value, "b0": b0.value, "b": b.value, "D": D.value, "S": S.value}


def ranmar_state(seed, stream_id, pair_counter):
    """The RANMAR state (L[W - 96 .. W], C[W]) of stream (seed, stream_id)
    at word W = 2 pair_counter, host only: a list of 98 integers."""
    out = (ctypes.c_uint32 * 98)()
    _check(lib().prngd_ranmar_state(seed, stream_id, pair_counter, out))
    return list(out)


def _map(m):
    return MAPS[m] if isinstance(m, str) else int(m)


def describe_map(generator, k, min, max, map):
    """(offset added to N, denominator, folded constant) of a map, host only."""
    off = ctypes.c_uint64()
    D = ctypes.c_uint64()
    S = ctypes.c_double()
    _check(lib().prngd_describe_map(_gen(generator), k, min, max, _map(map), ctypes.byref(off),
                                    ctypes.byref(D), ctypes.byref(S)))
    return {"n_offset": off.value, "D": D.value, "S": S.value}


def natural_range(generator, w):
    """(min, max) that prngd_create expects for a generator at resolution 2^-w."""
    g = _gen(generator)
    if g == MRG32K3A:
        return 1, M1
    return 0, (1 << w) - 1


class Generator:
    """A PRNGD stream handle: Algorithm 1's PRNGD(k, min, max) with a base
    generator and a seed, positioned at (stream_id, pair counter)."""

    def __init__(self, seed, generator="philox", w=32, k=None, min=None, max=None,
                 _handle=None, map=None, consume=None, words=None):
        g = _gen(generator)
        if k is None:
            k = 2.0 ** -w
        if min is None or max is None:
            lo, hi = natural_range(g, w)
            min = lo if min is None else min
            max = hi if max is None else max
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib().prngd_create(seed, g, k, min, max, ctypes.byref(h)))
        else:
            h = _handle
        self._h = h
        self.generator = g
        self.seed = seed
        self.k = k
        if map is not None:
            self.set_map(map)
        if consume is not None:
            self.set_consume(consume)
        if words is not None:
            self.set_arity(words)

    def set_arity(self, words):
        """Words combined per output: 2 (default) or 3 (the two-word method
        applied twice; the position then counts triples)."""
        _check(lib().prngd_set_arity(self.handle, int(words)))

    def get_arity(self):
        a = ctypes.c_uint32()
        _check(lib().prngd_get_arity(self.handle, ctypes.byref(a)))
        return a.value

    def set_consume(self, consume):
        """"pair" (default) or "single" (Algorithm 1: a rejected r1 consumes
        one word; the position then counts words)."""
        c = CONSUMES[consume] if isinstance(consume, str) else int(consume)
        _check(lib().prngd_set_consume(self.handle, c))

    def get_consume(self):
        c = ctypes.c_int()
        _check(lib().prngd_get_consume(self.handle, ctypes.byref(c)))
        return c.value

    def set_map(self, map):
        """Map of later outputs: "eq5" (default), "eq4" or "one_minus"."""
        _check(lib().prngd_set_map(self.handle, _map(map)))

    def get_map(self):
        m = ctypes.c_int()
        _check(lib().prngd_get_map(self.handle, ctypes.byref(m)))
        return m.value

    @classmethod
    def many(cls, seed, count, generator="philox", w=32, first_stream_id=0, k=None,
             min=None, max=None):
        """`count` generators on consecutive substreams of one seed, all at
        pair counter 0, created without any GPU work."""
        g = _gen(generator)
        if k is None:
            k = 2.0 ** -w
        lo, hi = natural_range(g, w)
        min = lo if min is None else min
        max = hi if max is None else max
        arr = (ctypes.c_void_p * count)()
        _check(lib().prngd_create_many(seed, g, k, min, max, first_stream_id, count, arr))
        return [cls(seed, g, w=w, k=k, min=min, max=max, _handle=ctypes.c_void_p(arr[i]))
                for i in range(count)]

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("generator is closed")
        return self._h

    def fill(self, out, n=None, stream=None):
        ptr, n = _out_ptr(out, n)
        _check(lib().prngd_fill(self.handle, n, ptr, _stream_ptr(stream)))
        return out

    def fill_noalloc(self, out, n=None, stream=None):
        ptr, n = _out_ptr(out, n)
        _check(lib().prngd_fill_noalloc(self.handle, n, ptr, _stream_ptr(stream)))
        return out

    def set_position(self, stream_id, pair_counter, stream=None):
        _check(lib().prngd_set_position(self.handle, stream_id, pair_counter,
                                        _stream_ptr(stream)))

    def get_position(self, stream=None):
        sid = ctypes.c_uint32()
        ctr = ctypes.c_uint64()
        _check(lib().prngd_get_position(self.handle, ctypes.byref(sid), ctypes.byref(ctr),
                                        _stream_ptr(stream)))
        return sid.value, ctr.value

    def close(self):
        if self._h is not None:
            _check(lib().prngd_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _requests(pairs):
    reqs = (Request * len(pairs))()
    for i, item in enumerate(pairs):
        gen, out = item[0], item[1]
        n = item[2] if len(item) > 2 else None
        ptr, n = _out_ptr(out, n)
        reqs[i].h = gen.handle
        reqs[i].n = n
        reqs[i].out = ptr
    return reqs


def fill_batch(pairs, stream=None):
    """pairs: [(Generator, tensor) or (Generator, tensor, n), ...]; one launch."""
    reqs = _requests(pairs)
    _check(lib().prngd_fill_batch(reqs, len(pairs), _stream_ptr(stream)))


_REQUEST_DTYPE = None


def fill_batch_raw(handles, ns, ptrs, stream):
    """The same as fill_batch, from plain integers: handle addresses (the
    `.handle.value` of each Generator), output counts and device addresses
    of 8-byte aligned float64 buffers the caller keeps alive; `stream` is a
    hipStream_t address.  For request loops where per-request marshalling
    matters."""
    import numpy as np
    global _REQUEST_DTYPE
    if _REQUEST_DTYPE is None:
        _REQUEST_DTYPE = _request_dtype()
        assert _REQUEST_DTYPE.itemsize == ctypes.sizeof(Request)
    count = len(handles)
    arr = np.empty(count, dtype=_REQUEST_DTYPE)
    arr["h"] = handles
    arr["n"] = ns
    arr["out"] = ptrs
    _check(lib().prngd_fill_batch(arr.ctypes.data_as(ctypes.POINTER(Request)), count, stream))


def fill_raw(handle, n, ptr, stream):
    """prngd_fill from plain integers (see fill_batch_raw)."""
    _check(lib().prngd_fill(ctypes.c_void_p(handle), n, ctypes.c_void_p(ptr), stream))


class Plan:
    """A resident batch replayed through a HIP graph."""

    def __init__(self, pairs):
        reqs = _requests(pairs)
        p = ctypes.c_void_p()
        _check(lib().prngd_plan_create(reqs, len(pairs), ctypes.byref(p)))
        self._p = p
        self._keep = pairs

    def launch(self, stream=None):
        _check(lib().prngd_plan_launch(self._p, _stream_ptr(stream)))

    def close(self):
        if self._p is not None:
            _check(lib().prngd_plan_destroy(self._p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PATHS = {"auto": 0, "ordered": 1, "speculative": 2, "speculative-hold": 3,
         "speculative-wave": 4, "speculative-chunk": 5, "counted": 6}


def set_tuning(generator, w, pairs_per_lane=0, blocks_per_cu=0, store_mode=0, slack_mode=0,
               block_threads=0, seq_max_tiles=0, path=0):
    """Launch shape for (generator, w); `path` is 0/"auto", 1/"ordered",
    2/"speculative", 3/"speculative-hold", 4/"speculative-wave" (single
    fills in 128-pair chunks) or 5/"speculative-chunk" (batches in chunks of
    pairs_per_lane / 2 windows of 128 pairs, one per wave; single fills as
    4) or 6/"counted" (single fills: count the accepted pairs of every
    512-pair chunk, scan, produce each chunk at its offset)."""
    path = PATHS.get(path, path)
    t = Tuning(pairs_per_lane, blocks_per_cu, store_mode, slack_mode, block_threads,
               seq_max_tiles, path)
    _check(lib().prngd_set_tuning(_gen(generator), w, ctypes.byref(t)))


def reset_tuning(generator, w):
    _check(lib().prngd_set_tuning(_gen(generator), w, None))


def get_tuning(generator, w):
    t = Tuning()
    _check(lib().prngd_get_tuning(_gen(generator), w, ctypes.byref(t)))
    return {"pairs_per_lane": t.pairs_per_lane, "blocks_per_cu": t.blocks_per_cu,
            "store_mode": t.store_mode, "slack_mode": t.slack_mode,
            "block_threads": t.block_threads, "seq_max_tiles": t.seq_max_tiles,
            "path": t.path}


# ------------------------------------------------------------------ probes
def _probe(rc):
    if rc != 0:
        raise PrngdError(rc, f"probe failed with code {rc}")


def probe_write(out, stream=None):
    """Coalesced 16-byte stores over all of `out` (float64 CUDA tensor)."""
    ptr, n = _out_ptr(out, None)
    _probe(lib().prngd_probe_write(ptr, n, _stream_ptr(stream)))


def probe_copy(dst, src, stream=None):
    """Copy float64 CUDA tensor `src` into `dst` (same length, disjoint)."""
    pd, n = _out_ptr(dst, None)
    ps, ns = _out_ptr(src, None)
    if n != ns:
        raise PrngdError(ERR_INVALID_ARGUMENT, "probe_copy: lengths differ")
    _probe(lib().prngd_probe_copy(pd, ps, n, _stream_ptr(stream)))


def probe_philox(sink, blocks, stream=None):
    """`blocks` Philox4x32-10 blocks folded into `sink` (int32 CUDA tensor)."""
    _probe(lib().prngd_probe_philox(sink.data_ptr(), sink.numel(), blocks, _stream_ptr(stream)))


def probe_set_spin_limit(polls):
    """Polls of a look-back wait before it reports a stall, for launches
    planned from now on (0: the default).  For tests of the stall path."""
    lib().prngd_probe_set_spin_limit(polls)


def probe_philox_store(out, stream=None):
    """Philox pairs mapped and stored to all of `out`, no acceptance test."""
    ptr, n = _out_ptr(out, None)
    _probe(lib().prngd_probe_philox_store(ptr, n, _stream_ptr(stream)))
