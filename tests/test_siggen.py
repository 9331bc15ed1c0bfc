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


def test_own_transcendentals_match_libm():
    rng = np.random.default_rng(3)
    for x in np.concatenate([rng.random(5000), 2.0 ** -rng.uniform(0, 33, 2000),
                             [2.0 ** -33, 0.5, 1.0 - 2.0 ** -33, 0.7071067811865476]]):
        want = math.log(x)
        got = siggen._test_ln(float(x))
        assert abs(got - want) <= 4e-16 * max(abs(want), 1e-300) + 1e-300 or \
            abs(got - want) <= 2.3e-16, (x, got, want)
    for n in (1, 2, 3, 7, 1000, 1536, 4096, 6000, 1 << 20, 1 << 31):
        for j in sorted(set(list(range(0, min(n, 64))) +
                            [int(v) for v in rng.integers(0, n, 300)])):
            c, s = siggen._test_turn(j, n)
            a = 2.0 * math.pi * (j / n)
            assert abs(c - math.cos(a)) < 2e-15 and abs(s - math.sin(a)) < 2e-15, (n, j)


def test_instruction_set_versions_are_bitwise_equal():
    sigs = [workloads.long_signal(), workloads.large_signal(),
            siggen.Signal(seed=5, seg_len=6000, sigma=0.5, tones=[(7, 0.3, 1.0)],
                          chirp_amp=0.7)]
    try:
        for sig in sigs:
            ref = None
            for cap in (0, 1, 2):
                siggen.set_isa(cap)
                got = sig.samples(3, 100001).view(np.uint32)
                if ref is None:
                    ref = got
                assert np.array_equal(ref, got), cap
            e = []
            for cap in (0, 1, 2):
                siggen.set_isa(cap)
                e.append(siggen.segment_energy(sig.samples(0, 4 * 6000).reshape(4, 6000)))
            assert np.array_equal(e[0], e[1]) and np.array_equal(e[0], e[2])
    finally:
        siggen.set_isa(2)


def test_noise_sample_is_box_muller_of_its_draw_words():
    """Samples 2j and 2j+1 take words (0, 1) and (2, 3) of Philox draw j
    (counter (j, 0, stream, 0), key = seed)."""
    seed, stream, sigma = 0x1234567890ABCDEF, 7, 1.5
    x = siggen.Signal(seed=seed, seg_len=1, sigma=sigma, stream=stream).samples(0, 64)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for j in (0, 1, 5, 31):
        r = siggen.philox4x32_10([j, 0, stream, 0], key)
        for h in (0, 1):
            u1 = (r[2 * h] + 0.5) / 2.0 ** 32
            u2 = (r[2 * h + 1] + 0.5) / 2.0 ** 32
            rad = sigma * math.sqrt(-2.0 * math.log(u1))
            want = complex(rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2))
            got = complex(x[2 * j + h])
            assert abs(got - want) <= 1e-6 * abs(want) + 1e-7, (j, h, got, want)


def test_segment_energies():
    sig = siggen.Signal(seed=11, seg_len=3000, sigma=1.0, tones=[(5, 0.5, 0.3)])
    x, e = sig.segments_with_energy(2, 7)
    assert np.array_equal(x, sig.segments(2, 7))
    want = (x.real.astype(np.float64) ** 2 + x.imag.astype(np.float64) ** 2).sum(axis=1)
    assert np.all(np.abs(e - want) <= 1e-13 * want)
    assert np.all(np.abs(siggen.segment_energy(x) - want) <= 1e-13 * want)
    # a segment length that is not a multiple of the 8-sample lanes
    y = sig.samples(0, 5 * 1001).reshape(5, 1001)
    wy = (y.real.astype(np.float64) ** 2 + y.imag.astype(np.float64) ** 2).sum(axis=1)
    assert np.all(np.abs(siggen.segment_energy(y) - wy) <= 1e-13 * wy)


def test_checked_chunk_callbacks_on_the_host():
    """The streamed run's producer and consumer, called directly on one host
    buffer (the consumer sees the producer's samples): input and output
    energies agree, the first and last segment of each chunk are kept, and
    a wrong chunk size or index is refused."""
    import ctypes
    n, spc, chunks = 256, 6, 3
    sig = siggen.Signal(seed=3, seg_len=n, sigma=1.0, chirp_amp=0.5)
    fill, drain, src, chk = sig.checked_chunk_source(spc, chunks, first_seg=4)
    FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                          ctypes.c_void_p, ctypes.c_uint64)
    f, d = FN(fill), FN(drain)
    buf = np.zeros(spc * n, np.complex64)
    u = ctypes.cast(ctypes.pointer(src), ctypes.c_void_p)
    for c in range(chunks):
        assert f(u, c, buf.ctypes.data, buf.nbytes) == 0
        assert np.array_equal(buf.reshape(spc, n), sig.segments(4 + c * spc, spc))
        assert d(u, c, buf.ctypes.data, buf.nbytes) == 0
        assert np.array_equal(chk.saved_out[c, 0], buf[:n])
        assert np.array_equal(chk.saved_out[c, 1], buf[-n:])
    assert np.allclose(chk.energy_in, chk.energy_out, rtol=1e-13, atol=0)
    assert np.all(chk.energy_in > 0)
    assert f(u, chunks, buf.ctypes.data, buf.nbytes) != 0
    assert d(u, 0, buf.ctypes.data, buf.nbytes - 8) != 0
