"""Helpers of the GPU tests: device-side bit comparison against oracle
outputs, arenas of request outputs, and a progress line before each GPU
step (test infrastructure)."""
import sys

import numpy as np

DEV = "cuda:0"
NAN_BITS = 0x7FF8DEADBEEF0001      # a pattern the kernels never write


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def upload(arrays, total=None):
    """Concatenate float64 numpy arrays into one device tensor."""
    import torch
    total = sum(len(a) for a in arrays) if total is None else total
    dst = torch.empty(total, dtype=torch.float64, device=DEV)
    off = 0
    for a in arrays:
        dst[off:off + len(a)].copy_(torch.from_numpy(np.ascontiguousarray(a)))
        off += len(a)
    return dst


def assert_device_bits_equal(got, expect, what, offsets=None):
    """got, expect: float64 device tensors of one length, compared as bit
    patterns.  offsets (optional, host int64 array of request starts plus
    the end) name the first request that differs."""
    import torch
    g = got.view(torch.int64)
    e = expect.view(torch.int64)
    if torch.equal(g, e):
        return
    bad = torch.nonzero(g != e)
    count = int(bad.numel())
    i = int(bad[0, 0]) if count else -1
    where = ""
    if offsets is not None and i >= 0:
        r = int(np.searchsorted(offsets, i, side="right") - 1)
        where = f", request {r} output {i - int(offsets[r])}"
    raise AssertionError(f"{what}: {count} mismatching outputs, first at {i}{where}: "
                         f"{float(got[i])!r} vs {float(expect[i])!r}")


class Arena:
    """One device tensor holding every request's output, back to back,
    pre-filled with a pattern the kernels never write."""

    def __init__(self, sizes):
        import torch
        self.sizes = [int(n) for n in sizes]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.total = int(self.offsets[-1])
        self.buf = torch.empty(max(self.total, 1), dtype=torch.float64, device=DEV)
        self.views = [self.buf[int(self.offsets[i]):int(self.offsets[i + 1])]
                      for i in range(len(self.sizes))]

    def poison(self):
        import torch
        self.buf.view(torch.int64).fill_(NAN_BITS)

    @property
    def data(self):
        return self.buf[:self.total]
