"""Recipes of the synthetic workloads (all seeded, all synthetic).

The paper measured on an unnamed 16 GB signal file and targets files over
1 TB (Sec. III-IV); no such file exists here, so seeded synthetic signals of
the same structure stand in: a long complex-FP32 signal cut into fixed-length
segments.

Seeds are ``BASE_SEED + workload index``.  Within a workload, Philox
streams separate the independent draws:

  stream 0   noise samples of the signal
  stream 1   tone bins           stream 2   tone amplitudes
  stream 3   tone phases         stream 4   segment lengths (uneven batch)
  stream 5   arrival gaps        stream 6   job sizes      stream 7  job lengths
  stream 1000 + j   noise of serving job j (tones: 2000 + j, 3000 + j)
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

from . import Signal, distinct_bins, normal, uniform

BASE_SEED = 0x14076915

# (segment_len, batch) of the fixed-length workloads
SMALL = dict(name="fwd_c2c_n1024_b1024", seg_len=1024, batch=1024)
LARGE = dict(name="fwd_c2c_n4096_b262144", seg_len=4096, batch=262144)
LONG = dict(name="fwd_c2c_n1048576_b32768_streamed", seg_len=1 << 20,
            batch=32768, chunk_segments=512)
UNEVEN_LENGTHS = (256, 1000, 1536, 4096, 6000, 16384, 65536)
UNEVEN = dict(name="uneven_200000_segments", n_segments=200000)
SERVING_LENGTHS = (1024, 4096, 65536, 1 << 20)


def small_signal() -> Signal:
    """1024-point segments: Gaussian noise sigma=1 per I/Q plus 3 unit
    amplitude bin-centred tones (distinct seeded bins, phase 0)."""
    seed = BASE_SEED + 0
    n = SMALL["seg_len"]
    bins = distinct_bins(seed, 1, n, 3)
    return Signal(seed=seed, seg_len=n, sigma=1.0, stream=0,
                  tones=[(b, 1.0, 0.0) for b in bins])


def large_signal() -> Signal:
    """4096-point segments: noise sigma=1 plus 8 bin-centred tones with
    log-uniform amplitudes in [1e-3, 1] and uniform phases in [0, 2 pi)."""
    seed = BASE_SEED + 1
    n = LARGE["seg_len"]
    bins = distinct_bins(seed, 1, n, 8)
    amps = 10.0 ** (-3.0 + 3.0 * uniform(seed, 2, 0, 8))
    phs = 2.0 * math.pi * uniform(seed, 3, 0, 8)
    return Signal(seed=seed, seg_len=n, sigma=1.0, stream=0,
                  tones=[(b, float(a), float(p))
                         for b, a, p in zip(bins, amps, phs)])


def long_signal() -> Signal:
    """2^20-point segments: noise sigma=1 plus the unit linear chirp
    exp(i pi n^2 / N) in every segment (sweeps the band once)."""
    seed = BASE_SEED + 2
    return Signal(seed=seed, seg_len=LONG["seg_len"], sigma=1.0, stream=0,
                  chirp_amp=1.0)


def uneven_lengths(n_segments: int = UNEVEN["n_segments"]) -> np.ndarray:
    """Segment lengths drawn i.i.d. uniformly from UNEVEN_LENGTHS."""
    u = uniform(BASE_SEED + 3, 4, 0, n_segments)
    idx = np.minimum((u * len(UNEVEN_LENGTHS)).astype(np.int64),
                     len(UNEVEN_LENGTHS) - 1)
    return np.asarray(UNEVEN_LENGTHS, dtype=np.int64)[idx]


def uneven_signal() -> Signal:
    """Noise sigma=1; segments of uneven length are packed back to back,
    so the signal is addressed by global sample index only."""
    return Signal(seed=BASE_SEED + 3, seg_len=1, sigma=1.0, stream=0)


@dataclass
class Job:
    """One serving request: ``n_seg`` segments of ``seg_len`` samples that
    arrive at ``arrival_s`` (seconds from the start)."""
    index: int
    arrival_s: float
    seg_len: int
    n_seg: int

    @property
    def samples(self) -> int:
        return self.seg_len * self.n_seg


def serving_jobs(rate_hz: float, n_jobs: int, seed_offset: int = 0,
                 cap_samples: int = 1 << 30) -> List[Job]:
    """Poisson arrivals at ``rate_hz``; job size lognormal(median 2^22,
    sigma 1.5) samples capped at 2^30; segment length uniform over
    SERVING_LENGTHS; n_seg = max(1, floor(size / seg_len))."""
    seed = BASE_SEED + 4 + (seed_offset << 8)
    gaps = -np.log(uniform(seed, 5, 0, n_jobs)) / rate_hz
    z = normal(seed, 6, 0, n_jobs)
    size = np.minimum(np.round(np.exp(math.log(2.0 ** 22) + 1.5 * z)),
                      cap_samples)
    u = uniform(seed, 7, 0, n_jobs)
    lidx = np.minimum((u * len(SERVING_LENGTHS)).astype(np.int64),
                      len(SERVING_LENGTHS) - 1)
    t = np.cumsum(gaps)
    jobs = []
    for j in range(n_jobs):
        n = SERVING_LENGTHS[lidx[j]]
        jobs.append(Job(j, float(t[j]), n, max(1, int(size[j]) // n)))
    return jobs


def job_signal(job: Job, seed_offset: int = 0) -> Signal:
    """Payload of a serving job: noise sigma=1 plus 2 bin-centred tones."""
    seed = BASE_SEED + 4 + (seed_offset << 8)
    bins = distinct_bins(seed, 2000 + job.index, job.seg_len, 2)
    amps = 10.0 ** (-3.0 + 3.0 * uniform(seed, 3000 + job.index, 0, 2))
    return Signal(seed=seed, seg_len=job.seg_len, sigma=1.0,
                  stream=1000 + job.index,
                  tones=[(b, float(a), 0.0) for b, a in zip(bins, amps)])
