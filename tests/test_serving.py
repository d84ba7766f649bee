"""The serving loop, the autotuner and the batched-vs-plain comparison.

CPU: the first-fit arena the serving loop allocates outputs from.
GPU: every request served in a mix of concurrent batches (and by the plain
baseline) equals the same request filled alone, bit for bit, in each
client's arrival order; the autotuner's choice leaves the output bytes
unchanged.
"""
import random
import sys

import numpy as np
import pytest

import oracle as O


def test_arena_first_fit_and_coalescing():
    torch = pytest.importorskip("torch")
    from paper_1401_8230_amd.serving import Arena
    a = Arena(1000, device="cpu")
    rng = random.Random(5)
    live = {}
    for step in range(3000):
        if live and (rng.random() < 0.5 or len(live) > 40):
            off = rng.choice(list(live))
            a.release(off, live.pop(off))
        else:
            n = rng.randint(1, 120)
            off = a.alloc(n)
            if off is None:
                assert sum(ln for _, ln in a.free) < n or max(ln for _, ln in a.free) < n
                continue
            # no overlap with a live block
            for o, ln in live.items():
                assert off + n <= o or o + ln <= off
            assert 0 <= off and off + n <= 1000
            live[off] = n
        assert a.used == sum(live.values())
        # free list sorted, disjoint, coalesced
        for (o1, l1), (o2, l2) in zip(a.free, a.free[1:]):
            assert o1 + l1 < o2
    for off, n in list(live.items()):
        a.release(off, n)
    assert a.free == [(0, 1000)] and a.used == 0


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _check_against_alone(served, clients):
    refs = {c: O.PRNGD(O.GEN_PHILOX, 32, seed=42, stream=c) for c in range(clients)}
    for r in sorted(served, key=lambda r: r.rid):
        expect = refs[r.client].fill(r.n)
        got = np.ascontiguousarray(r.out)
        if not np.array_equal(got.view(np.uint64), expect.view(np.uint64)):
            bad = int(np.flatnonzero(got.view(np.uint64) != expect.view(np.uint64))[0])
            raise AssertionError(f"request {r.rid} (client {r.client}, n={r.n}): first "
                                 f"mismatch at {bad}")


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_served_requests_equal_the_same_requests_alone(mode):
    pytest.importorskip("torch")
    from paper_1401_8230_amd import serving, workloads
    clients = 48
    trace = workloads.poisson_trace(count=500, rate=5e4, lo=1e2, hi=2e5, clients=clients,
                                    rng_seed=11)
    note(f"serving {mode}: {len(trace)} requests")
    # a small budget makes requests wait for memory as well as for clients
    res = serving.run_trace(trace, mode=mode, clients=clients, budget_bytes=4e6 * 8,
                            streams=3, keep_outputs=True)
    served = res["served"]
    assert len(served) == len(trace)
    assert all(r.done is not None and r.done >= r.arrival for r in served)
    _check_against_alone(served, clients)
    assert res["p50_ms"] <= res["p99_ms"]


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_served_large_requests_sampled(mode):
    # the serving trace's own shape: 1024 clients, sizes log-uniform in
    # [1e2, 1e8]; every request's first and last 512 outputs and all outputs
    # of every 40th request and of the largest ones are checked against the
    # oracle walking each client's stream through its requests in order
    pytest.importorskip("torch")
    from concurrent.futures import ThreadPoolExecutor

    import oracle_parallel as OP
    from paper_1401_8230_amd import serving, workloads
    clients = 1024
    trace = workloads.poisson_trace(count=400, rate=4e3, lo=1e2, hi=1e8, clients=clients,
                                    rng_seed=777)
    note(f"serving {mode}, large: {len(trace)} requests, {sum(a.n for a in trace)} outputs")
    res = serving.run_trace(trace, mode=mode, clients=clients, budget_bytes=12e9,
                            keep_outputs="sample")
    served = res["served"]
    assert len(served) == len(trace)
    assert max(r.n for r in served) > 5 * 10**7
    by_client = {}
    for r in sorted(served, key=lambda r: r.rid):
        by_client.setdefault(r.client, []).append(r)

    def check(client):
        ref = O.PRNGD(O.GEN_PHILOX, 32, seed=42, stream=client)
        for r in by_client[client]:
            expect = ref.fill(r.n)
            kept = r.out
            for part, want in (("head", expect[:512]), ("tail", expect[-512:]),
                               ("full", expect if kept["full"] is not None else None)):
                if want is None:
                    continue
                got = np.ascontiguousarray(kept[part])
                if not np.array_equal(got.view(np.uint64), want.view(np.uint64)):
                    return f"request {r.rid} (client {client}, n={r.n}): {part} differs"
        return None

    with ThreadPoolExecutor(max_workers=OP.host_threads()) as pool:
        errors = [e for e in pool.map(check, list(by_client)) if e]
    assert not errors, errors[:3]


@pytest.mark.gpu
def test_autotuned_batch_keeps_bytes(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_1401_8230_amd import autotune, prngd, workloads
    reqs = workloads.uneven_batch(count=64, lo=1, hi=2e5, rng_seed=3)
    sizes = [r.n for r in reqs]
    outs = [torch.empty(n, dtype=torch.float64, device="cuda:0") for n in sizes]
    note("autotune 64 uneven requests")
    res = autotune.autotune_batch(sizes, outs, "philox", 32,
                                  cache_path=str(tmp_path / "tune.json"), reps=1)
    assert res["table"] and not res["from_cache"]
    again = autotune.autotune_batch(sizes, outs, "philox", 32,
                                    cache_path=str(tmp_path / "tune.json"))
    assert again["from_cache"] and again["tuning"] == res["tuning"]
    try:
        gens = [prngd.Generator(r.seed, "philox", w=32) for r in reqs]
        for g, r in zip(gens, reqs):
            g.set_position(r.stream_id, r.counter)
        prngd.fill_batch(list(zip(gens, outs)))
        torch.cuda.synchronize()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            expect = O.PRNGD(O.GEN_PHILOX, 32, seed=r.seed, stream=r.stream_id,
                             counter=r.counter).fill(r.n)
            assert np.array_equal(o.cpu().numpy().view(np.uint64), expect.view(np.uint64)), i
        for g in gens:
            g.close()
    finally:
        prngd.reset_tuning("philox", 32)


@pytest.mark.parametrize("gen,w", [("philox", 32), ("philox", 24), ("mixed", 32),
                                   ("mrg32k3a", 32)])
def test_autotune_candidates_are_valid_launch_shapes(gen, w):
    from paper_1401_8230_amd import autotune, prngd
    cands = autotune.candidates(gen, w)
    assert len(cands) >= 6
    paths = {c.get("path", 0) for c in cands}
    assert {1, 2} <= paths
    try:
        for c in cands:
            prngd.set_tuning(gen, w, **c)             # validated on the host
            t = prngd.get_tuning(gen, w)
            for k, v in c.items():
                assert t[k] == v, (k, c)
    finally:
        prngd.reset_tuning(gen, w)
