"""A continuous-batching request loop for PRNGD fills.

Clients ask for the next n outputs of their own stream.  Each client is a
handle whose position lives on the device and advances with every fill,
so the loop never reads positions back.  The loop

* queues arriving requests per client (a client's requests run in arrival
  order, at most one of them on the GPU at a time);
* admits queued requests while their outputs fit in the HBM budget (one
  preallocated arena, first-fit);
* launches every admitted request of a round as one batched fill on the
  next free HIP stream, so batches that arrive while others run overlap
  on the device;
* retires a batch when its event has completed, which frees its memory and
  its clients.

``mode="plain"`` serves the same trace one prngd_fill per request in
arrival order on one stream (first come, first served), the baseline.

Latency of a request = the host time its completion was observed minus its
scheduled arrival time.
"""
import bisect
import gc
import time
from collections import deque

from . import prngd


class Arena:
    """First-fit allocator over one float64 device tensor (offsets and
    lengths in elements)."""

    def __init__(self, elements, device="cuda:0"):
        import torch
        self.buf = torch.empty(int(elements), dtype=torch.float64, device=device)
        self.base = self.buf.data_ptr()
        self.size = int(elements)
        self.free = [(0, self.size)]          # sorted (offset, length)
        self.used = 0

    def alloc(self, n):
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                return off
        return None

    def release(self, off, n):
        self.used -= n
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # coalesce with the neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)

    def view(self, off, n):
        return self.buf[off:off + n]

    def address(self, off):
        return self.base + 8 * off


def kept_output(r, view, keep):
    """What a served request keeps of its output for checking: everything
    (keep=True), or with keep="sample" the first and last 512 outputs and
    all of them for every 40th request and for requests of 5e7 or more."""
    if keep == "sample":
        full = r.rid % 40 == 0 or r.n >= 5 * 10**7
        return {"head": view[:512].cpu().numpy(), "tail": view[-512:].cpu().numpy(),
                "full": view.cpu().numpy() if full else None}
    return view.cpu().numpy()


class Request:
    __slots__ = ("rid", "client", "n", "arrival", "done", "off", "out")

    def __init__(self, rid, client, n, arrival):
        self.rid = rid
        self.client = client
        self.n = n
        self.arrival = arrival
        self.done = None
        self.off = None
        self.out = None


class Server:
    """Continuous batching over `clients` handles (substreams 0..clients-1
    of `seed`) with an HBM budget of `budget_bytes` of outputs in flight."""

    def __init__(self, clients=1024, generator="philox", w=32, seed=42, budget_bytes=64e9,
                 streams=4, max_batch=512, keep_outputs=False):
        import torch
        self.gens = prngd.Generator.many(seed, clients, generator, w=w)
        self.hids = [g.handle.value for g in self.gens]
        self.arena = Arena(int(budget_bytes) // 8)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.sptrs = [st.cuda_stream for st in self.streams]
        self.events = [torch.cuda.Event() for _ in range(streams)]
        self.stream_busy = [None] * streams           # in-flight batch per stream
        self.queues = {}                              # client -> deque of requests
        self.order = deque()                          # clients with queued work, FIFO
        self.busy = set()                             # clients with a request on the GPU
        self.max_batch = max_batch
        self.keep = keep_outputs
        self.finished = []
        self.queued = 0                               # requests not yet launched
        self._warm_streams(generator, w)

    def _warm_streams(self, generator, w):
        """One small and one full-size batch on every stream, on scratch
        handles, so that each stream's workspace exists and is large enough
        before requests arrive."""
        import torch
        scratch = prngd.Generator.many(0x5EED, self.max_batch, generator, w=w)
        try:
            n_big = min(10**8, self.arena.size // 4)
            for s in self.streams:
                prngd.fill_batch([(scratch[0], self.arena.view(0, n_big)),
                                  (scratch[1], self.arena.view(n_big, n_big))], stream=s)
                prngd.fill_batch([(g, self.arena.view(i * 64, 64))
                                  for i, g in enumerate(scratch)], stream=s)
            torch.cuda.synchronize()
        finally:
            for g in scratch:
                g.close()

    def submit(self, req):
        if req.n * 8 > self.arena.size * 8:
            raise ValueError(f"request of {req.n} outputs exceeds the HBM budget")
        q = self.queues.get(req.client)
        if q is None:
            q = self.queues[req.client] = deque()
        if not q:
            self.order.append(req.client)
        q.append(req)
        self.queued += 1

    def _retire(self, now_fn):
        for i, b in enumerate(self.stream_busy):
            if b is None or not b[0].query():
                continue
            t = now_fn()
            for r in b[1]:
                r.done = t
                if self.keep:
                    r.out = kept_output(r, self.arena.view(r.off, r.n), self.keep)
                self.arena.release(r.off, r.n)
                self.busy.discard(r.client)
                self.finished.append(r)
            self.stream_busy[i] = None
            # clients freed by this batch may have queued work
            for r in b[1]:
                if self.queues.get(r.client):
                    self.order.append(r.client)

    def _admit(self):
        batch = []
        skipped = deque()
        while self.order and len(batch) < self.max_batch:
            c = self.order.popleft()
            q = self.queues.get(c)
            if not q or c in self.busy:
                continue                        # re-queued when its batch retires
            r = q[0]
            off = self.arena.alloc(r.n)
            if off is None:
                skipped.append(c)               # waits for memory; keeps its place
                continue
            q.popleft()
            self.queued -= 1
            r.off = off
            self.busy.add(c)
            batch.append(r)
        self.order.extendleft(reversed(skipped))
        return batch

    def step(self, now_fn):
        """Retire finished batches, then launch one new batch if a stream is
        free.  Returns True if anything happened."""
        before = len(self.finished)
        self._retire(now_fn)
        progressed = len(self.finished) != before
        try:
            slot = self.stream_busy.index(None)
        except ValueError:
            return progressed
        batch = self._admit()
        if not batch:
            return progressed
        if len(batch) == 1:
            # a round of one request: the plain fill, without batch marshalling
            r = batch[0]
            prngd.fill_raw(self.hids[r.client], r.n, self.arena.address(r.off), self.sptrs[slot])
        else:
            prngd.fill_batch_raw([self.hids[r.client] for r in batch], [r.n for r in batch],
                                 [self.arena.address(r.off) for r in batch], self.sptrs[slot])
        ev = self.events[slot]
        ev.record(self.streams[slot])
        self.stream_busy[slot] = (ev, batch)
        return True

    def idle(self):
        return self.queued == 0 and all(b is None for b in self.stream_busy)

    def close(self):
        import torch
        torch.cuda.synchronize()
        for g in self.gens:
            g.close()
        self.gens = []


class PlainServer:
    """The baseline: one prngd_fill per request, in arrival order, on one
    stream; memory from the same kind of budgeted arena."""

    def __init__(self, clients=1024, generator="philox", w=32, seed=42, budget_bytes=64e9,
                 keep_outputs=False):
        import torch
        self.gens = prngd.Generator.many(seed, clients, generator, w=w)
        self.hids = [g.handle.value for g in self.gens]
        self.arena = Arena(int(budget_bytes) // 8)
        self.stream = torch.cuda.Stream()
        self.sptr = self.stream.cuda_stream
        self.pool = []                           # retired events, reused
        self.waiting = deque()
        self.running = deque()                   # (event, request), in order
        self.keep = keep_outputs
        self.finished = []

    def submit(self, req):
        self.waiting.append(req)

    def step(self, now_fn):
        import torch
        progressed = False
        while self.running and self.running[0][0].query():
            ev, r = self.running.popleft()
            r.done = now_fn()
            if self.keep:
                r.out = kept_output(r, self.arena.view(r.off, r.n), self.keep)
            self.arena.release(r.off, r.n)
            self.pool.append(ev)
            self.finished.append(r)
            progressed = True
        while self.waiting:
            r = self.waiting[0]
            off = self.arena.alloc(r.n)
            if off is None:
                break                            # first come, first served
            self.waiting.popleft()
            r.off = off
            prngd.fill_raw(self.hids[r.client], r.n, self.arena.address(off), self.sptr)
            ev = self.pool.pop() if self.pool else torch.cuda.Event()
            ev.record(self.stream)
            self.running.append((ev, r))
            progressed = True
        return progressed

    def idle(self):
        return not self.running and not self.waiting

    def close(self):
        import torch
        torch.cuda.synchronize()
        for g in self.gens:
            g.close()
        self.gens = []


def percentile(values, q):
    if not values:
        return float("nan")
    v = sorted(values)
    k = (len(v) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def preload_kernels(generator="philox", w=32, sizes=(100, 10**4, 10**6, 3 * 10**7)):
    """Run every fill form a request loop may pick once, on scratch handles,
    so that no kernel is loaded for the first time while requests wait."""
    import torch
    gens = prngd.Generator.many(0x5EED, 2, generator, w=w)
    try:
        buf = torch.empty(2 * max(sizes), dtype=torch.float64, device="cuda:0")
        for n in sizes:
            gens[0].fill(buf[:n])
            prngd.fill_batch([(gens[0], buf[:n]), (gens[1], buf[n:2 * n])])
        torch.cuda.synchronize()
    finally:
        for g in gens:
            g.close()


def run_trace(trace, mode="batched", warmup=0, clients=1024, budget_bytes=64e9, streams=4,
              keep_outputs=False, log=None, server=None):
    """Replay `trace` (workloads.Arrival items) in real time.  Returns
    throughput over the measured requests (all after the first `warmup`)
    and latency percentiles in milliseconds; with keep_outputs the served
    requests (with host copies of their outputs) under "requests"."""
    import torch
    if server is None:
        if mode == "batched":
            server = Server(clients=clients, budget_bytes=budget_bytes, streams=streams,
                            keep_outputs=keep_outputs)
        else:
            server = PlainServer(clients=clients, budget_bytes=budget_bytes,
                                 keep_outputs=keep_outputs)
    reqs = [Request(i, a.client, a.n, a.t) for i, a in enumerate(trace)]
    preload_kernels()
    torch.cuda.synchronize()
    # a full garbage collection in the middle of the loop would stall it
    gc_was_enabled = gc.isenabled()
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    i = 0
    try:
        while i < len(reqs) or not server.idle():
            t = now()
            while i < len(reqs) and reqs[i].arrival <= t:
                server.submit(reqs[i])
                i += 1
            server.step(now)
    finally:
        if gc_was_enabled:
            gc.enable()
    measured = [r for r in reqs[warmup:]]
    lat = [(r.done - r.arrival) * 1e3 for r in measured]
    first = min(r.arrival for r in measured)
    last = max(r.done for r in measured)
    outputs = sum(r.n for r in measured)
    res = {
        "requests": len(measured),
        "outputs": outputs,
        "seconds": last - first,
        "value": outputs / (last - first),
        "unit": "accepted FP64 uniforms/s",
        "p50_ms": percentile(lat, 0.50),
        "p99_ms": percentile(lat, 0.99),
        "max_ms": max(lat),
        "offered_per_s": sum(r.n for r in measured) / (measured[-1].arrival - first)
        if len(measured) > 1 else float("nan"),
    }
    if keep_outputs:
        res["served"] = reqs
    server.close()
    return res
