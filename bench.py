"""Benchmark of the PRNGD fill on one MI355X.

Default workload: 2^16 independent Philox4x32-10 substreams of seed 42
(substream id in counter word 3), w = 32, 2^14 FP64 outputs each -- 2^30
outputs, 8 GiB written per step -- filled by one resident batch (the
request descriptors live in device memory, the persistent fill kernel is
replayed from a HIP graph).  A step is one such launch; every handle
advances, so every step produces new numbers.

Prints one JSON line: accepted FP64 uniforms per second, the roofline of
the fill kernel (HBM write bandwidth; 8 algorithmic bytes per output) and
the CPU oracle's rate on a bounded sample of the same workload.
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
KERNEL_SRC = os.path.join(ROOT, "paper_1401_8230_amd", "csrc", "prngd_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_many_streams.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--streams", type=int, default=1 << 16)
    ap.add_argument("--outputs-per-stream", type=int, default=1 << 14)
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-streams", type=int, default=16384)
    ap.add_argument("--calibrate", action="store_true",
                    help="after the timed steps, copy half of the output buffer onto the "
                         "other half once (the known-size kernel that scales HBM counters)")
    return ap.parse_args()


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from rocprofv3 counter runs, if they were taken
    on the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding of the fill is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1401_8230_amd import prngd

    torch.cuda.set_device(0)
    n = args.outputs_per_stream
    S = args.streams
    print(f"[bench] creating {S} handles", file=sys.stderr, flush=True)
    gens = prngd.Generator.many(args.seed, S, "philox", w=32)
    out = torch.empty(S * n, dtype=torch.float64, device="cuda:0")
    views = [out[i * n:(i + 1) * n] for i in range(S)]
    plan = prngd.Plan(list(zip(gens, views)))
    stream = torch.cuda.current_stream()
    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.launch(stream)
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        plan.launch(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = start.elapsed_time(stop) / 1e3
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)

    outputs = S * n
    step_s = gpu_s / args.steps
    value = outputs * args.steps / gpu_s
    achieved_gbs = outputs * BYTES_PER_OUTPUT / step_s / 1e9
    lo, hi = float(out.min()), float(out.max())
    if not (0.0 <= lo and hi < 1.0):
        raise SystemExit(f"outputs out of [0, 1): {lo} {hi}")
    if args.calibrate:
        half = outputs // 2
        prngd.probe_copy(out[half:2 * half], out[:half], stream)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {half * 8} bytes", file=sys.stderr, flush=True)
    plan.close()

    traffic = measured_traffic()
    result = {
        "metric": "accepted FP64 uniforms/s",
        "value": value,
        "unit": "accepted FP64 uniforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "wall_ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{S} Philox4x32-10 substreams of seed {args.seed}, w=32, "
                        f"{n} FP64 outputs each, one resident batch per step",
            "streams": S,
            "outputs_per_stream": n,
            "outputs_per_step": outputs,
            "launch": "persistent fill kernel replayed from a HIP graph",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(min(args.cpu_sample_streams, S), n, args.seed)
    for g in gens:
        g.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
