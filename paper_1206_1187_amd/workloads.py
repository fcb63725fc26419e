"""Seeded synthetic workloads for the alpha_{2,3} generator.

This module only draws inputs (seed indices, offsets, lengths, arrival
times) with numpy's ``default_rng``; it performs none of the generator's
arithmetic, so the oracle and the HIP path can both be fed from it.

The paper measures a single stream of 2^28 doubles (inferred from Table 2)
and prints no dataset; every workload here is synthetic:

* ``plain_single``  -- seed index 3^33+100, 2^20 consecutive outputs.
* ``plain_bulk``    -- one seed index drawn with seed 1 over the valid range
  (Algorithm BB step 1), 2^30 f64 outputs plus a 2^28 u64 run.
* ``skip_stress``   -- 65,536 offsets drawn with seed 2 over [0, period),
  4,096 f64 outputs each, with offsets forced next to the period wrap.
* ``batched``       -- 10,000 streams (seed 3), lengths log-uniform in
  [1, 2^22].
* ``served``        -- Poisson arrivals (seed 4) at 20k req/s for 10 s,
  sizes log-uniform in [256, 2^24], over 1,024 client streams.
"""
from dataclasses import dataclass

import numpy as np

#: 3^33: index range and period bounds of the input domain (Algorithm BB).
MODULUS = 3 ** 33
#: Period of the sequence, 2 * 3^32 (Section 2).
PERIOD = 2 * 3 ** 32
#: Valid starting indices, inclusive (Algorithm BB step 1).
INDEX_MIN = MODULUS + 100
INDEX_MAX = 2 ** 53


@dataclass
class PlainCase:
    name: str
    index: int
    count_f64: int
    count_u64: int


def plain_single() -> PlainCase:
    return PlainCase("plain_single", INDEX_MIN, 1 << 20, 1 << 20)


def plain_bulk() -> PlainCase:
    rng = np.random.default_rng(1)
    a = int(rng.integers(INDEX_MIN, INDEX_MAX, endpoint=True, dtype=np.int64))
    return PlainCase("plain_bulk", a, 1 << 30, 1 << 28)


def skip_offsets(n: int = 65536, length: int = 4096) -> np.ndarray:
    """Offsets into the stream of seed index 3^33+100 (uint64)."""
    rng = np.random.default_rng(2)
    off = rng.integers(0, PERIOD, n, dtype=np.int64).astype(np.uint64)
    # Uniform draws practically never land next to the wrap; force some there.
    off[0] = 0
    off[1] = PERIOD - 1
    k = min(64, n - 2)
    for j in range(k):
        off[n - 1 - j] = PERIOD - 1 - j * 64
    return off


@dataclass
class BatchedCase:
    indices: np.ndarray  # uint64 seed index per stream
    lengths: np.ndarray  # uint64 outputs per stream


def batched(n_streams: int = 10000, max_log2: int = 22) -> BatchedCase:
    rng = np.random.default_rng(3)
    idx = rng.integers(INDEX_MIN, INDEX_MAX, n_streams, endpoint=True, dtype=np.int64)
    u = rng.uniform(0.0, max_log2 * np.log(2.0), n_streams)
    lens = np.clip(np.floor(np.exp(u)), 1, 2 ** max_log2).astype(np.uint64)
    return BatchedCase(idx.astype(np.uint64), lens)


@dataclass
class ServedTrace:
    stream_indices: np.ndarray  # uint64 seed index per client stream
    t_arrive: np.ndarray        # float64 seconds, nondecreasing
    stream_id: np.ndarray       # int32
    count: np.ndarray           # uint64 outputs per request


def served(rate: float = 20000.0, duration: float = 10.0, n_streams: int = 1024,
           lo: int = 256, hi: int = 1 << 24) -> ServedTrace:
    rng = np.random.default_rng(4)
    seeds = rng.integers(INDEX_MIN, INDEX_MAX, n_streams, endpoint=True, dtype=np.int64)
    # Draw gaps in blocks until the horizon is passed.
    n_guess = int(rate * duration * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, n_guess)
    t = np.cumsum(gaps)
    while t[-1] < duration:
        more = rng.exponential(1.0 / rate, n_guess)
        t = np.concatenate([t, t[-1] + np.cumsum(more)])
    t = t[t < duration]
    n = t.size
    sizes = np.clip(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), n))), lo, hi)
    sid = rng.integers(0, n_streams, n).astype(np.int32)
    return ServedTrace(seeds.astype(np.uint64), t, sid, sizes.astype(np.uint64))
