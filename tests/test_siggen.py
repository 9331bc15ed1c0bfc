"""The seeded generator: Philox known answers, determinism, chunk
independence, and that the synthesised tones and chirp are what their
recipes say (checked through the oracle's spectra)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import siggen
from siggen import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    g = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in g["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        out = [int(h, 16) for h in v["out"]]
        assert list(siggen.philox4x32_10(ctr, key)) == out


def test_determinism_and_chunk_independence():
    s = siggen.Signal(seed=123, seg_len=64, sigma=1.0,
                      tones=[(5, 0.5, 1.0)], chirp_amp=0.25)
    whole = s.samples(0, 10000)
    assert np.array_equal(whole, s.samples(0, 10000, threads=1))
    for a, n in [(0, 1), (17, 333), (4096, 5904), (9999, 1)]:
        assert np.array_equal(s.samples(a, n), whole[a:a + n])
    assert np.array_equal(s.segments(3, 2), whole[3 * 64:5 * 64].reshape(2, 64))
    other = siggen.Signal(seed=124, seg_len=64, sigma=1.0).samples(0, 100)
    assert not np.array_equal(other, siggen.Signal(seed=123, seg_len=64,
                                                   sigma=1.0).samples(0, 100))


def test_noise_statistics():
    x = siggen.Signal(seed=9, seg_len=1, sigma=1.0).samples(0, 1 << 20)
    for comp in (x.real, x.imag):
        assert abs(comp.mean()) < 5e-3
        assert abs(comp.astype(np.float64).var() - 1.0) < 5e-3
    u = siggen.uniform(1, 2, 0, 100000)
    assert u.min() > 0 and u.max() < 1 and abs(u.mean() - 0.5) < 5e-3
    z = siggen.normal(1, 2, 0, 100000)
    assert abs(z.mean()) < 2e-2 and abs(z.var() - 1) < 2e-2


@pytest.mark.parametrize("n", [1024, 4096])
def test_tones_are_bin_centred(n):
    tones = [(3, 1.0, 0.0), (n // 2 + 1, 0.01, 2.0), (n - 1, 0.5, -1.0)]
    s = siggen.Signal(seed=1, seg_len=n, sigma=0.0, tones=tones)
    X = oracle.fft_recursive(s.segments(5, 2), n)   # segment 5 and 6
    for seg in X:
        want = np.zeros(n, complex)
        for b, a, p in tones:
            want[b] = n * a * np.exp(1j * p)
        # float32 rounding of the time samples only
        assert np.linalg.norm(seg - want) < 1e-6 * np.linalg.norm(want)


def test_chirp_matches_gauss_sum():
    n = 4096
    s = siggen.Signal(seed=1, seg_len=n, sigma=0.0, chirp_amp=1.0)
    X = oracle.fft_recursive(s.segments(1, 1), n)[0]
    k = np.arange(n)
    want = math.sqrt(n) * np.exp(1j * np.pi / 4) * \
        np.exp(-1j * np.pi * ((k * k) % (2 * n)) / n)
    assert np.linalg.norm(X - want) < 1e-6 * np.linalg.norm(want)


def test_workload_recipes():
    s = workloads.small_signal()
    assert s.seg_len == 1024 and len(s.tones) == 3
    assert len({t[0] for t in s.tones}) == 3
    assert all(t[1] == 1.0 and t[2] == 0.0 for t in s.tones)
    big = workloads.large_signal()
    amps = [t[1] for t in big.tones]
    assert len(big.tones) == 8 and min(amps) >= 1e-3 and max(amps) <= 1
    assert all(0 <= t[2] < 2 * math.pi for t in big.tones)
    lens = workloads.uneven_lengths(70000)
    vals, cnt = np.unique(lens, return_counts=True)
    assert tuple(vals) == workloads.UNEVEN_LENGTHS
    assert cnt.min() > 9000
    assert np.array_equal(lens[:100], workloads.uneven_lengths(100))
    jobs = workloads.serving_jobs(100.0, 2000)
    assert all(j.n_seg >= 1 and j.samples <= 1 << 30 for j in jobs)
    arr = np.array([j.arrival_s for j in jobs])
    assert np.all(np.diff(arr) > 0)
    assert abs(len(jobs) / arr[-1] - 100.0) < 10.0
    med = np.median([j.n_seg * j.seg_len for j in jobs])
    assert 2 ** 21 < med < 2 ** 23
