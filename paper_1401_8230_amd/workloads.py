"""Seeded synthetic workloads (request lists) shared by the tests and the
benchmark.  Only inputs live here -- seeds, substreams, start positions and
sizes -- none of the PRNGD arithmetic.

The paper measures on no dataset; these recipes stand in for the
workloads the method is meant for (many independent Monte Carlo streams,
uneven request sizes, arrivals over time).
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Request:
    seed: int
    stream_id: int
    counter: int
    n: int


def many_streams(num_streams=1 << 16, n_each=1 << 14, seed=42):
    """Independent substreams 0..num_streams-1 of one seed, each filled from
    pair 0 with n_each outputs."""
    return [Request(seed, s, 0, n_each) for s in range(num_streams)]


def uneven_batch(count=4096, lo=1e3, hi=1e7, rng_seed=4096, max_counter=1 << 48):
    """`count` requests with sizes log-uniform in [lo, hi], each with its own
    seed and substream and a random start position (odd and mid-block
    starts, low-word carries included)."""
    rng = np.random.default_rng(rng_seed)
    u = rng.random(count)
    sizes = np.floor(10.0 ** (np.log10(lo) + (np.log10(hi) - np.log10(lo)) * u)).astype(np.int64)
    seeds = rng.integers(0, 2**63, size=count, dtype=np.int64)
    counters = rng.integers(0, max_counter, size=count, dtype=np.int64)
    return [Request(int(seeds[i]), i, int(counters[i]), int(sizes[i])) for i in range(count)]


@dataclass(frozen=True)
class Arrival:
    t: float          # seconds since the start of the trace
    client: int
    n: int


def poisson_trace(count=20000, rate=2e4, lo=1e2, hi=1e8, clients=1024, rng_seed=20000):
    """Open-loop Poisson arrivals at `rate` per second with log-uniform sizes
    in [lo, hi]; request r belongs to client r mod `clients`."""
    rng = np.random.default_rng(rng_seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    times = np.cumsum(gaps) - gaps[0]
    u = rng.random(count)
    sizes = np.floor(10.0 ** (np.log10(lo) + (np.log10(hi) - np.log10(lo)) * u)).astype(np.int64)
    return [Arrival(float(times[i]), i % clients, int(sizes[i])) for i in range(count)]
