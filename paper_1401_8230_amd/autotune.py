"""Autotuner for the launch shape of batched PRNGD fills.

For a batch shape (request sizes and their output buffers) it times every
candidate launch shape -- threads per workgroup, pairs per lane (outputs
per lane), store width, the ordered or speculative path, and how many
tiles a request may have and still be produced whole by one workgroup
(workgroups per stream) -- as a resident plan replayed on the GPU, keeps
the fastest, applies it with ``prngd.set_tuning`` and remembers it in a
JSON cache keyed by the device and the batch shape.  Tuning never changes
output bytes, so the choice is purely a matter of speed.

The timing runs on scratch handles (their own seed), never on the
caller's handles: autotuning consumes no random numbers of the caller's
streams.
"""
import json
import math
import os

from . import prngd

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "prngd_autotune.json")


def _philox_shapes():
    return [(256, 4), (256, 8), (256, 16), (256, 32), (512, 8), (512, 16), (1024, 16)]


def candidates(generator, w):
    """Launch shapes worth timing for (generator, w), as set_tuning keyword
    dictionaries."""
    g = prngd._gen(generator)
    out = []
    if g in (prngd.MRG32K3A, prngd.PHILOX_X1_MRG32K3A_X2):
        for ppl in (4, 8, 16):
            for seq in (0, 1 << 20):
                out.append({"block_threads": 256, "pairs_per_lane": ppl, "seq_max_tiles": seq,
                            "path": 1})
            out.append({"block_threads": 256, "pairs_per_lane": ppl, "path": 2})
        return out
    for ppl in (2, 4, 8):
        # the chunk form: one chunk of ppl / 2 windows of 128 pairs per wave
        out.append({"pairs_per_lane": ppl, "path": 5})
    for threads, ppl in _philox_shapes():
        for store_mode in (0, 2):
            for path in (2, 3):
                out.append({"block_threads": threads, "pairs_per_lane": ppl,
                            "store_mode": store_mode, "path": path})
            for seq in (0, 1 << 20):
                out.append({"block_threads": threads, "pairs_per_lane": ppl,
                            "store_mode": store_mode, "path": 1, "seq_max_tiles": seq})
    return out


def device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{p.multi_processor_count}CU"


def shape_key(generator, w, sizes):
    total = sum(sizes)
    big = max(sizes) if sizes else 0
    return (f"{prngd._gen(generator)}|w{w}|count{len(sizes)}|"
            f"total2^{round(math.log2(max(total, 1)), 1)}|max2^{round(math.log2(max(big, 1)), 1)}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(sizes, outs, generator, w, tuning, warmup=1, reps=3, seed=0xA070, stream=None):
    """Seconds per replay of a resident plan over scratch handles with the
    given launch shape."""
    import torch
    prngd.set_tuning(generator, w, **tuning)
    gens = prngd.Generator.many(seed, len(sizes), generator, w=w)
    plan = None
    try:
        plan = prngd.Plan([(g, o, n) for g, o, n in zip(gens, outs, sizes)])
        s = stream or torch.cuda.current_stream()
        for _ in range(warmup):
            plan.launch(s)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            plan.launch(s)
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b) / 1e3 / reps
    finally:
        if plan is not None:
            plan.close()
        for g in gens:
            g.close()


def autotune_batch(sizes, outs, generator="philox", w=32, cache_path=None, retune=False,
                   warmup=1, reps=3, log=None):
    """Pick and apply the fastest launch shape for a batch of `sizes`
    outputs written to `outs` (float64 CUDA tensors, one per request).
    Returns {"tuning": ..., "seconds": ..., "from_cache": bool, "table": [...]}."""
    cache_path = cache_path or os.environ.get("PRNGD_AUTOTUNE_CACHE", DEFAULT_CACHE)
    key = device_key() + "|" + shape_key(generator, w, sizes)
    cache = _load(cache_path)
    if not retune and key in cache:
        best = cache[key]
        prngd.set_tuning(generator, w, **best["tuning"])
        return {"tuning": best["tuning"], "seconds": best["seconds"], "from_cache": True,
                "table": []}
    table = []
    for cand in candidates(generator, w):
        try:
            sec = time_plan(sizes, outs, generator, w, cand, warmup=warmup, reps=reps)
        except prngd.PrngdError as e:
            if log:
                log(f"[autotune] {cand}: {e}")
            continue
        table.append((sec, cand))
        if log:
            log(f"[autotune] {cand}: {sec * 1e3:.3f} ms")
    if not table:
        prngd.reset_tuning(generator, w)
        raise RuntimeError("autotune: no candidate launch shape ran")
    sec, best = min(table, key=lambda x: x[0])
    prngd.set_tuning(generator, w, **best)
    cache[key] = {"tuning": best, "seconds": sec}
    _store(cache_path, cache)
    return {"tuning": best, "seconds": sec, "from_cache": False,
            "table": [{"seconds": s, "tuning": c} for s, c in table]}
