"""Benchmark of the PRNGD fill on one MI355X.

Headline workload: 2^16 independent Philox4x32-10 substreams of seed 42
(substream id in counter word 3), w = 32, 2^14 FP64 outputs each -- 2^30
outputs, 8 GiB written per step -- filled by one resident batch (the
request descriptors live in device memory, the fill is replayed from a
HIP graph).  A step is one such launch; every handle advances, so every
step produces new numbers.

Prints one JSON line: accepted FP64 uniforms per second, the roofline of
the fill kernel (HBM write bandwidth; 8 algorithmic bytes per output), the
CPU oracle's rate on a bounded sample of the same workload, and, unless
--headline-only, more measurements on the same GPU:

* single_stream: large fills of one stream, each step one prngd_fill that
  continues the stream -- Philox4x32-10 at w = 32 with 2^30 outputs per
  fill (8 GiB), and 2^28 outputs per fill (2 GiB) of the mixed
  Philox/MRG32k3a generator, of MRG32k3a alone and of Philox at w = 24 --
  each with its own roofline and a bounded oracle sample;

* batched_vs_plain: 4096 requests with log-uniform sizes in [1e3, 1e7],
  each with its own seed, substream and start position, as one autotuned
  resident batch versus 4096 plain prngd_fill calls (and versus plain
  calls that each wait for their result), with identical output bytes;
* serving: a Poisson trace of fill requests (2e4 per second, sizes
  log-uniform in [1e2, 1e8], 1024 clients with device-resident positions)
  served by the continuous-batching loop under a 64 GB HBM budget, against
  the same trace served one plain fill at a time: throughput, p50, p99;
  and both loops at saturation (arrivals far faster than service), with
  the trace's sizes and with small requests.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
BYTES_PER_OUTPUT = 8           # one FP64 written per accepted pair
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_many_streams.json")
TRAFFIC_FILE_SINGLE = os.path.join(ROOT, "profiles", "traffic_single_stream.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--streams", type=int, default=1 << 16)
    ap.add_argument("--outputs-per-stream", type=int, default=1 << 14)
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--workload", choices=["many_streams", "single"], default="many_streams",
                    help="timed step: the resident many-streams batch (default), or one "
                         "prngd_fill of --single-outputs outputs of one Philox stream")
    ap.add_argument("--single-outputs", type=int, default=1 << 30)
    ap.add_argument("--generator", choices=["philox", "mrg32k3a", "mixed", "ranmar"],
                    default="philox",
                    help="base generator of the single-stream workload (mixed: x1 from "
                         "Philox4x32-10, x2 from MRG32k3a)")
    ap.add_argument("--width", type=int, default=32,
                    help="w of the single-stream workload (Philox only below 32)")
    ap.add_argument("--consume", choices=["pair", "single"], default="pair",
                    help="what a rejected x1 consumes (single: Algorithm 1's loop)")
    ap.add_argument("--map", choices=["eq5", "eq4", "one_minus"], default="eq5",
                    help="output map: Eq. (5), Eq. (4) / Algorithm 1's Z, or 1 - z")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-streams", type=int, default=16384)
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the batched-vs-plain and serving measurements")
    ap.add_argument("--single-steps", type=int, default=20,
                    help="timed fills of each single-stream leg")
    ap.add_argument("--no-single-legs", action="store_true",
                    help="skip the single-stream legs of the default run")
    ap.add_argument("--uneven-steps", type=int, default=5)
    ap.add_argument("--serving-requests", type=int, default=20000)
    ap.add_argument("--calibrate", action="store_true",
                    help="after the timed steps, copy half of the output buffer onto the "
                         "other half once (the known-size kernel that scales HBM counters)")
    return ap.parse_args()


def kernel_hash():
    from paper_1401_8230_amd._build import kernel_source_hash
    return kernel_source_hash()


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch from rocprofv3 counter runs, if they were taken
    on the current kernel source; otherwise None."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(streams, n_each, seed):
    import oracle as O
    t0 = time.perf_counter()
    total = 0
    for s in range(streams):
        o = O.PRNGD(O.GEN_PHILOX, 32, seed=seed, stream=s)
        o.fill(n_each)
        total += n_each
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "accepted FP64 uniforms/s", "cores": 1,
            "kind": "oracle",
            "sample": f"substreams 0..{streams - 1} of the same workload, {n_each} outputs "
                      f"each ({total} outputs, {dt:.1f} s, one thread)"}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_all_cores(streams, n_each, seed, max_threads=16):
    """The same oracle on every host core given to this process (at most
    max_threads), one independent substream per task; the oracle's C calls
    run without the interpreter lock."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(ncpu, max_threads))

    def one(s):
        O.PRNGD(O.GEN_PHILOX, 32, seed=seed, stream=s).fill(n_each)
        return n_each

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        total = sum(pool.map(one, range(streams)))
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "accepted FP64 uniforms/s", "cores": threads,
            "kind": "oracle", "nproc": ncpu, "cpu_model": host_cpu_model(),
            "sample": f"substreams 0..{streams - 1} of the same workload, {n_each} outputs "
                      f"each ({total} outputs, {dt:.1f} s, {threads} threads)"}


def cpu_baseline_single(n, seed, generator="philox", w=32):
    import oracle as O
    gen = {"philox": O.GEN_PHILOX, "mrg32k3a": O.GEN_MRG32K3A, "mixed": O.GEN_MIXED,
           "ranmar": O.GEN_RANMAR}[generator]
    t0 = time.perf_counter()
    O.PRNGD(gen, w, seed=seed, stream=0).fill(n)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "accepted FP64 uniforms/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {n} outputs of the same stream ({dt:.1f} s, one thread)"}


def timed(fn, steps, stream):
    """Seconds per call of fn over `steps` calls, HIP events on `stream`."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3 / steps


def per_step(fn, steps, stream):
    """Median, min and max milliseconds of `steps` further calls of fn, each
    between its own pair of HIP events on `stream` (after the timed region,
    so that it does not disturb it)."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(steps):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    return {"median": ms[len(ms) // 2], "min": ms[0], "max": ms[-1], "steps": steps}


def run_many_streams(args, result):
    import torch
    from paper_1401_8230_amd import prngd
    n = args.outputs_per_stream
    S = args.streams
    log(f"many streams: creating {S} handles")
    gens = prngd.Generator.many(args.seed, S, "philox", w=32)
    for g in gens:
        if args.consume != "pair":
            g.set_consume(args.consume)
        if args.map != "eq5":
            g.set_map(args.map)
    out = torch.empty(S * n, dtype=torch.float64, device="cuda:0")
    views = [out[i * n:(i + 1) * n] for i in range(S)]
    plan = prngd.Plan(list(zip(gens, views)))
    stream = torch.cuda.current_stream()
    log("many streams: warmup")
    for _ in range(args.warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = timed(lambda: plan.launch(stream), args.steps, stream)
    wall = time.perf_counter() - t0
    log(f"many streams: timed {args.steps} steps, {step_s * 1e3:.3f} ms per step")
    dist = per_step(lambda: plan.launch(stream), args.steps, stream)
    outputs = S * n
    lo, hi = float(out.min()), float(out.max())
    if not (0.0 <= lo and hi < 1.0):
        raise SystemExit(f"outputs out of [0, 1): {lo} {hi}")
    if args.calibrate:
        half = outputs // 2
        prngd.probe_copy(out[half:2 * half], out[:half], stream)
        torch.cuda.synchronize()
        log(f"calibration copy of {half * 8} bytes")
    plan.close()
    for g in gens:
        g.close()
    del out, views
    achieved_gbs = outputs * BYTES_PER_OUTPUT / step_s / 1e9
    result.update({
        "value": outputs / step_s,
        "ms_per_step": step_s * 1e3,
        "wall_ms_per_step": wall / args.steps * 1e3,
        "step_ms": dist,
        "config": {
            "workload": f"{S} Philox4x32-10 substreams of seed {args.seed}, w=32, "
                        f"{n} FP64 outputs each, one resident batch per step"
                        + ("" if args.consume == "pair" and args.map == "eq5" else
                           f", consume={args.consume}, map={args.map}"),
            "streams": S,
            "outputs_per_stream": n,
            "outputs_per_step": outputs,
            "launch": "resident batch replayed from a HIP graph",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            # the counters were taken on the default form (pair consumption, Eq. (5))
            "traffic": measured_traffic() if args.consume == "pair" and args.map == "eq5"
            else None,
        },
    })


GENERATOR_NAMES = {"philox": "Philox4x32-10", "mrg32k3a": "MRG32k3a",
                   "mixed": "Philox4x32-10 (x1) and MRG32k3a (x2)", "ranmar": "RANMAR"}


def measured_leg_traffic(gen, w, n):
    """Committed HBM counters of one single-stream leg, if taken on the
    current kernel source."""
    name = f"traffic_single_{gen}_w{w}_n{n}.json"
    if gen == "philox" and w == 32 and n == 1 << 30:
        return measured_traffic(TRAFFIC_FILE_SINGLE)
    return measured_traffic(os.path.join(ROOT, "profiles", name))


def single_leg(gen, w, n, steps, warmup, seed=42, map="eq5", consume="pair", calibrate=False):
    """One stream of `gen` at resolution 2^-w (seed, substream 0): each step
    is one prngd_fill of n outputs continuing the stream."""
    import torch
    from paper_1401_8230_amd import prngd
    g = prngd.Generator(seed, gen, w=w, map=map,
                        consume=None if consume == "pair" else consume)
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        g.fill(out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = timed(lambda: g.fill(out, stream=stream), steps, stream)
    wall = time.perf_counter() - t0
    log(f"single stream {gen} w={w}: {n} outputs, {step_s * 1e3:.3f} ms per fill")
    dist = per_step(lambda: g.fill(out, stream=stream), steps, stream)
    lo, hi = float(out.min()), float(out.max())
    if not (0.0 <= lo and hi <= 1.0):
        raise SystemExit(f"outputs out of range: {lo} {hi}")
    if calibrate:
        half = n // 2
        prngd.probe_copy(out[half:2 * half], out[:half], stream)
        torch.cuda.synchronize()
    g.close()
    del out
    achieved_gbs = n * BYTES_PER_OUTPUT / step_s / 1e9
    default_form = consume == "pair" and map == "eq5"
    return {
        "value": n / step_s,
        "unit": "accepted FP64 uniforms/s",
        "ms_per_step": step_s * 1e3,
        "wall_ms_per_step": wall / steps * 1e3,
        "steps": steps,
        "step_ms": dist,
        "workload": f"one {GENERATOR_NAMES[gen]} stream of seed {seed}, w={w}, {n} FP64 "
                    f"outputs per fill, each fill continuing the stream"
                    + ("" if default_form else f", consume={consume}, map={map}"),
        "outputs_per_step": n,
        "launch": "prngd_fill",
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": measured_leg_traffic(gen, w, n) if default_form else None},
    }


# the single-stream legs of the default run: (generator, w, outputs per fill)
SINGLE_LEGS = [("philox", 32, 1 << 30), ("mixed", 32, 1 << 28), ("mrg32k3a", 32, 1 << 28),
               ("philox", 24, 1 << 28), ("ranmar", 24, 1 << 28)]


def run_single(args, result):
    """--workload single: the headline is one stream of --generator at w = --width."""
    leg = single_leg(args.generator, args.width, args.single_outputs, args.steps, args.warmup,
                     seed=args.seed, map=args.map, consume=args.consume,
                     calibrate=args.calibrate)
    result.update({
        "value": leg["value"],
        "ms_per_step": leg["ms_per_step"],
        "wall_ms_per_step": leg["wall_ms_per_step"],
        "step_ms": leg["step_ms"],
        "config": {"workload": leg["workload"], "outputs_per_step": leg["outputs_per_step"],
                   "launch": "prngd_fill (speculative fill and its repair pass)"},
        "roofline": leg["roofline"],
    })


def run_single_legs(args):
    legs = {}
    for gen, w, n in SINGLE_LEGS:
        leg = single_leg(gen, w, n, args.single_steps, args.warmup, seed=args.seed)
        if not args.no_cpu_baseline:
            leg["cpu_baseline"] = cpu_baseline_single(min(n, 1 << 22), args.seed, gen, w)
        legs[f"{gen}_w{w}_n{n}"] = leg
    return legs


def run_uneven(args):
    """4096 uneven requests: autotuned resident batch vs plain fills."""
    import torch
    from paper_1401_8230_amd import autotune, prngd, workloads
    reqs = workloads.uneven_batch()
    sizes = [r.n for r in reqs]
    total = sum(sizes)
    log(f"uneven batch: {len(reqs)} requests, {total} outputs ({total * 8 / 1e9:.1f} GB)")
    arena = torch.empty(total, dtype=torch.float64, device="cuda:0")
    outs, off = [], 0
    for n in sizes:
        outs.append(arena[off:off + n])
        off += n
    tune = autotune.autotune_batch(sizes, outs, "philox", 32, retune=True)
    log(f"uneven batch: autotuned {tune['tuning']} ({tune['seconds'] * 1e3:.3f} ms)")
    gens = [prngd.Generator(r.seed, "philox", w=32) for r in reqs]
    for g, r in zip(gens, reqs):
        g.set_position(r.stream_id, r.counter)
    stream = torch.cuda.current_stream()

    # bit-identity: one batched launch (autotuned shape) and one round of
    # plain fills (library defaults) from the same start positions, compared
    # output by output on the device (a copy of the batched arena is kept)
    plan = prngd.Plan(list(zip(gens, outs)))
    plan.launch(stream)
    torch.cuda.synchronize()
    batched_copy = arena.clone()
    batched_ends = [g.get_position()[1] for g in gens]
    plan.close()
    prngd.reset_tuning("philox", 32)
    for g, r in zip(gens, reqs):
        g.set_position(r.stream_id, r.counter)
    for g, o in zip(gens, outs):
        g.fill(o, stream=stream)
    torch.cuda.synchronize()
    identical = bool(torch.equal(batched_copy.view(torch.int64), arena.view(torch.int64))) and \
        batched_ends == [g.get_position()[1] for g in gens]
    del batched_copy
    log(f"uneven batch: batched and plain outputs and end positions identical: {identical}")

    # the resident batch is built in the autotuned shape; plain fills keep
    # the library defaults
    prngd.set_tuning("philox", 32, **tune["tuning"])
    plan = prngd.Plan(list(zip(gens, outs)))
    prngd.reset_tuning("philox", 32)
    plan.launch(stream)
    batched_s = timed(lambda: plan.launch(stream), args.uneven_steps, stream)
    plan.close()
    log(f"uneven batch: batched {batched_s * 1e3:.3f} ms per step")

    def plain_round():
        for g, o in zip(gens, outs):
            g.fill(o, stream=stream)
    plain_round()
    plain_s = timed(plain_round, args.uneven_steps, stream)
    log(f"uneven batch: plain {plain_s * 1e3:.3f} ms per step")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, o in zip(gens, outs):
        g.fill(o, stream=stream)
        stream.synchronize()
    sync_s = time.perf_counter() - t0
    log(f"uneven batch: plain with a wait per request {sync_s * 1e3:.3f} ms per step")
    for g in gens:
        g.close()
    del arena, outs
    gbs = total * BYTES_PER_OUTPUT / batched_s / 1e9
    return {
        "workload": f"{len(reqs)} requests, sizes log-uniform in [1e3, 1e7], own seed, "
                    f"substream and start position each",
        "outputs_per_step": total,
        "batched": {"value": total / batched_s, "ms_per_step": batched_s * 1e3,
                    "hbm_frac": gbs / HBM_PEAK_GBS, "tuning": tune["tuning"]},
        "plain": {"value": total / plain_s, "ms_per_step": plain_s * 1e3},
        "plain_wait_each": {"value": total / sync_s, "ms_per_step": sync_s * 1e3},
        "speedup_vs_plain": plain_s / batched_s,
        "speedup_vs_plain_wait_each": sync_s / batched_s,
        "outputs_identical": identical,
        "unit": "accepted FP64 uniforms/s",
    }


def run_serving(args):
    from paper_1401_8230_amd import serving, workloads
    trace = workloads.poisson_trace(count=args.serving_requests + 1000)
    log(f"serving: {len(trace)} requests (first 1000 warm up)")
    batched = serving.run_trace(trace, mode="batched", warmup=1000, log=log)
    log(f"serving: batched p50 {batched['p50_ms']:.3f} ms p99 {batched['p99_ms']:.3f} ms")
    plain = serving.run_trace(trace, mode="plain", warmup=1000, log=log)
    log(f"serving: plain p50 {plain['p50_ms']:.3f} ms p99 {plain['p99_ms']:.3f} ms")
    # the same loops at saturation: arrivals far faster than either can
    # serve, once with the trace's sizes and once with small requests
    sat = {}
    for name, lo, hi, count in (("sizes_1e2_1e8", 1e2, 1e8, 4000),
                                ("sizes_1e2_1e4", 1e2, 1e4, 20000)):
        tr = workloads.poisson_trace(count=count, rate=1e8, lo=lo, hi=hi, rng_seed=7)
        b = serving.run_trace(tr, mode="batched")
        p = serving.run_trace(tr, mode="plain")
        log(f"serving at saturation ({name}): batched {b['value']:.3e}/s, "
            f"plain {p['value']:.3e}/s")
        sat[name] = {"requests": count, "batched": b, "plain": p,
                     "throughput_ratio": b["value"] / p["value"]}
    return {
        "workload": "Poisson arrivals at 2e4 requests/s, sizes log-uniform in [1e2, 1e8], "
                    "1024 clients, HBM budget 64 GB",
        "batched": batched,
        "plain": plain,
        "throughput_ratio": batched["value"] / plain["value"],
        "p99_ratio": plain["p99_ms"] / batched["p99_ms"],
        "saturated": sat,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the fill runs "
              "on one GPU; independent streams and requests would shard across GPUs with no "
              "communication", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    result = {
        "metric": "accepted FP64 uniforms/s",
        "value": None,
        "unit": "accepted FP64 uniforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
    }
    if args.workload == "single":
        run_single(args, result)
    else:
        run_many_streams(args, result)
    if not args.headline_only and not args.no_single_legs and args.workload != "single":
        result["single_stream"] = run_single_legs(args)
    if not args.headline_only:
        result["batched_vs_plain"] = run_uneven(args)
        result["serving"] = run_serving(args)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        if args.workload == "single":
            result["cpu_baseline"] = cpu_baseline_single(min(args.single_outputs, 1 << 28),
                                                         args.seed, args.generator, args.width)
        else:
            result["cpu_baseline"] = cpu_baseline(
                min(args.cpu_sample_streams, args.streams), args.outputs_per_stream, args.seed)
            if not args.headline_only:
                log("cpu baseline, all cores")
                result["cpu_baseline_all_cores"] = cpu_baseline_all_cores(
                    args.streams, args.outputs_per_stream, args.seed)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
