"""Pins of the FP64 oracle against what mathematics fixes.

Each check is chosen so that a plausible slip in the oracle fails it:
a wrong exponent sign moves a tone's spike to bin N-k0; a dropped or
mis-indexed term breaks agreement with the hand-written small DFT matrices,
with numpy's pocketfft and between the two independent routines; a wrong
twiddle index breaks the shift theorem and the chirp closed form.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import FORWARD, INVERSE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ROUTINES = [oracle.dft_direct, oracle.fft_recursive]


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def close(a, b, tol=1e-12):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    scale = max(np.linalg.norm(b), 1.0)
    return np.linalg.norm(a - b) <= tol * scale


# --- hand-written DFT matrices of tiny lengths (textbook values) -----------

@pytest.mark.parametrize("f", ROUTINES)
def test_tiny_lengths_by_hand(f):
    x = np.array([1 + 2j, -3 + 0.5j, 0.25 - 1j, 2 + 2j])
    # N = 1: identity
    assert close(f(x[:1], 1), x[:1])
    # N = 2: [a + b, a - b] both directions
    a, b = x[0], x[1]
    assert close(f(x[:2], 2, FORWARD), [a + b, a - b])
    assert close(f(x[:2], 2, INVERSE), [a + b, a - b])
    # N = 3 with w = exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2
    w = complex(-0.5, -math.sqrt(3) / 2)
    x3 = x[:3]
    want = [x3.sum(), x3[0] + w * x3[1] + w * w * x3[2],
            x3[0] + w * w * x3[1] + w * x3[2]]
    assert close(f(x3, 3, FORWARD), want)
    wc = w.conjugate()
    want_inv = [x3.sum(), x3[0] + wc * x3[1] + wc * wc * x3[2],
                x3[0] + wc * wc * x3[1] + wc * x3[2]]
    assert close(f(x3, 3, INVERSE), want_inv)
    # N = 4: forward matrix rows [1,1,1,1],[1,-i,-1,i],[1,-1,1,-1],[1,i,-1,-i]
    M = np.array([[1, 1, 1, 1], [1, -1j, -1, 1j], [1, -1, 1, -1],
                  [1, 1j, -1, -1j]])
    assert close(f(x, 4, FORWARD), M @ x)
    assert close(f(x, 4, INVERSE), M.conj() @ x)


# --- the two independent routines agree; numpy (pocketfft, FP64) agrees ---

SIZES = list(range(1, 65)) + [97, 125, 243, 256, 1000, 1024, 1536, 4096, 6000]


@pytest.mark.parametrize("n", SIZES)
def test_direct_vs_recursive_vs_numpy(n):
    rng = np.random.default_rng(1000 + n)
    batch = 3 if n <= 1536 else 1
    x = crandn(rng, batch, n)
    for d in (FORWARD, INVERSE):
        a = oracle.dft_direct(x, n, d)
        b = oracle.fft_recursive(x, n, d)
        lib = np.fft.fft(x, axis=-1) if d == FORWARD else \
            np.fft.ifft(x, axis=-1) * n
        assert oracle.rel_l2(a, b).max() < 1e-12, (n, d)
        assert oracle.rel_l2(b, lib).max() < 1e-12, (n, d)


@pytest.mark.parametrize("n", [7 * 64, 11 * 9, 13 * 25, 49])
def test_other_primes_fall_back_to_definition(n):
    rng = np.random.default_rng(n)
    x = crandn(rng, 2, n)
    assert oracle.rel_l2(oracle.fft_recursive(x, n),
                         np.fft.fft(x, axis=-1)).max() < 1e-12


def test_long_segment_against_numpy():
    n = 1 << 20
    rng = np.random.default_rng(7)
    x = crandn(rng, 1, n)
    assert oracle.rel_l2(oracle.fft_recursive(x, n),
                         np.fft.fft(x, axis=-1)).max() < 1e-12


# --- closed forms ----------------------------------------------------------

@pytest.mark.parametrize("n", [8, 1000, 1024, 4096, 6000])
@pytest.mark.parametrize("d", [FORWARD, INVERSE])
def test_impulse(n, d):
    for n0 in (0, 1, n // 3, n - 1):
        x = np.zeros(n, complex)
        x[n0] = 1.0
        k = np.arange(n)
        want = np.exp(d * 2j * np.pi * ((k * n0) % n) / n)
        for f in ROUTINES:
            assert close(f(x, n, d), want), (f.__name__, n0)


@pytest.mark.parametrize("n", [12, 1000, 4096])
def test_constant(n):
    c = 0.75 - 0.5j
    want = np.zeros(n, complex)
    want[0] = n * c
    for f in ROUTINES:
        for d in (FORWARD, INVERSE):
            assert close(f(np.full(n, c), n, d), want)


@pytest.mark.parametrize("n", [30, 1024, 1536, 4096, 6000])
def test_bin_tone_single_spike(n):
    k0 = (7 * n) // 13
    A = 0.3 + 0.4j
    t = np.arange(n)
    x = A * np.exp(2j * np.pi * ((k0 * t) % n) / n)
    fwd = np.zeros(n, complex)
    fwd[k0] = n * A                # forward: spike at +k0
    inv = np.zeros(n, complex)
    inv[(n - k0) % n] = n * A      # inverse: the same tone lands at -k0
    for f in ROUTINES:
        assert close(f(x, n, FORWARD), fwd)
        assert close(f(x, n, INVERSE), inv)


@pytest.mark.parametrize("n", [16, 1024, 4096, 1 << 20])
def test_alternating_and_chirp(n):
    t = np.arange(n, dtype=np.int64)
    alt = np.where(t % 2 == 0, 1.0, -1.0).astype(complex)
    want = np.zeros(n, complex)
    want[n // 2] = n
    f = oracle.fft_recursive
    assert close(f(alt, n), want)
    # unit chirp exp(i pi n^2 / N), N even:
    #   X[k] = sqrt(N) e^{i pi/4} e^{-i pi k^2 / N}  (quadratic Gauss sum)
    chirp = np.exp(1j * np.pi * ((t * t) % (2 * n)) / n)
    want = math.sqrt(n) * np.exp(1j * np.pi / 4) * \
        np.exp(-1j * np.pi * ((t * t) % (2 * n)) / n)
    assert close(f(chirp, n), want, 1e-11)
    if n <= 4096:
        assert close(oracle.dft_direct(chirp, n), want, 1e-11)


# --- invariants ------------------------------------------------------------

@pytest.mark.parametrize("n", [60, 1000, 1024, 6000])
def test_parseval_linearity_shift_symmetry_roundtrip(n):
    rng = np.random.default_rng(n)
    x = crandn(rng, n)
    y = crandn(rng, n)
    f = oracle.fft_recursive
    X = f(x, n)[0]
    Y = f(y, n)[0]
    # Parseval: sum |X|^2 = N sum |x|^2
    assert abs(np.sum(abs(X) ** 2) - n * np.sum(abs(x) ** 2)) < \
        1e-12 * n * np.sum(abs(x) ** 2)
    # linearity
    a, b = 2 - 1j, -0.5 + 3j
    assert close(f(a * x + b * y, n)[0], a * X + b * Y)
    # shift theorem: x[(t - m) mod N] <-> X[k] e^{-2 pi i k m / N}
    m = n // 7 + 1
    k = np.arange(n)
    assert close(f(np.roll(x, m), n)[0],
                 X * np.exp(-2j * np.pi * ((k * m) % n) / n))
    # real input: X[N - k] = conj(X[k])
    R = f(x.real.astype(complex), n)[0]
    assert close(R[(-k) % n], R.conj())
    # round trip: IFFT(FFT(x)) = N x
    assert close(f(X, n, INVERSE)[0], n * x)


def test_segments_are_independent_and_ordered():
    # a segment's spectrum depends on that segment alone and lands at the
    # same position (Sec. III: records keyed by offset, outputs by position)
    n, b = 256, 9
    rng = np.random.default_rng(3)
    x = crandn(rng, b, n)
    f = oracle.fft_recursive
    X = f(x, n)
    x2 = x.copy()
    x2[4] += crandn(rng, n)
    X2 = f(x2, n)
    assert np.array_equal(np.delete(X, 4, 0), np.delete(X2, 4, 0))
    assert not np.array_equal(X[4], X2[4])
    perm = rng.permutation(b)
    assert np.array_equal(f(x[perm], n), X[perm])
    for s in range(b):
        assert np.array_equal(f(x[s], n)[0], X[s])


# --- metric, tolerance, argument checks -------------------------------------

def test_rel_l2_and_tolerance():
    r = np.array([[1 + 0j, 0], [0, 0]])
    y = np.array([[1 + 1e-3j, 0], [0, 0]])
    e = oracle.rel_l2(y, r)
    assert abs(e[0] - 1e-3) < 1e-15 and e[1] == 0.0
    y[1, 0] = 1e-30
    assert np.isinf(oracle.rel_l2(y, r)[1])
    assert oracle.tolerance(4096) == pytest.approx(6e-6)
    assert oracle.tolerance(1000) == pytest.approx(5e-7 * math.log2(1000))
    assert oracle.tolerance(1) == pytest.approx(5e-7)


def test_bad_arguments():
    x = np.zeros(8, complex)
    with pytest.raises(ValueError):
        oracle.fft_recursive(x, 3)
    with pytest.raises(ValueError):
        oracle.fft_recursive(x, 8, 0)
    with pytest.raises(TypeError):
        oracle.fft_recursive(np.zeros(8), 8)


def test_float32_input_is_upcast_exactly():
    rng = np.random.default_rng(5)
    x32 = crandn(rng, 2, 64).astype(np.complex64)
    assert np.array_equal(oracle.fft_recursive(x32, 64),
                          oracle.fft_recursive(x32.astype(np.complex128), 64))


# --- the paper's segmentation arithmetic (Sec. III) --------------------------

def test_paper_record_arithmetic():
    g = json.load(open(os.path.join(GOLDEN, "paper_record_arithmetic.json")))
    n, bps = g["segment_len"], g["bytes_per_real_sample"]
    assert n * bps == g["record_bytes"]
    assert oracle.record_count(g["file_bytes"], n, bps) == g["records"]
    assert oracle.block_count(g["file_bytes"], g["block_bytes"]) == g["blocks"]
    assert oracle.record_offset(1, n, bps) == g["record_bytes"]
    # the complex64 records used here are twice as wide
    assert oracle.record_count(g["file_bytes"], n, 8) == g["records"] // 2
    assert oracle.record_offset(5, n, 8, base=64) == 64 + 5 * 8192


# --- overlapping, windowed segments -----------------------------------------

def _hann(n):
    # periodic Hann window 0.5 - 0.5 cos(2 pi j / n)
    return 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n) / n)


@pytest.mark.parametrize("n,hop,k0", [(64, 16, 5), (60, 7, 0), (32, 32, 31)])
def test_short_time_hann_tone_closed_form(n, hop, k0):
    """Frame s of exp(2 pi i k0 m / n) starts with phase exp(2 pi i k0 s hop / n);
    times the periodic Hann window its spectrum is n/2 at k0 and -n/4 at
    k0 +- 1 (mod n), all times that phase, and zero elsewhere."""
    frames_n = 9
    m = np.arange((frames_n - 1) * hop + n)
    x = np.exp(2j * np.pi * k0 * m / n)
    y = oracle.short_time(x, n, hop, frames_n, _hann(n))
    for s in range(frames_n):
        ph = np.exp(2j * np.pi * k0 * s * hop / n)
        want = np.zeros(n, dtype=np.complex128)
        want[k0] += 0.5 * n * ph
        want[(k0 + 1) % n] += -0.25 * n * ph
        want[(k0 - 1) % n] += -0.25 * n * ph
        assert np.max(np.abs(y[s] - want)) < 1e-9 * n


def test_frames_brute_force_and_disjoint_reduction():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    w = rng.uniform(0.1, 1.0, 8)
    f = oracle.frames(x, 8, 3, 15, w)
    for s in range(15):
        for j in range(8):
            assert f[s, j] == x[3 * s + j] * w[j]
    # hop == n, no window: the disjoint records of the plain path
    y = oracle.short_time(x[:48], 8, 8, 6)
    assert np.array_equal(y, oracle.fft_recursive(x[:48].astype(np.complex128), 8))
    # inverse direction is the plain inverse of each windowed frame
    yi = oracle.short_time(x, 8, 5, 9, w, INVERSE)
    assert np.allclose(yi, np.fft.ifft(oracle.frames(x, 8, 5, 9, w), axis=1) * 8)


def test_frames_bad_arguments():
    x = np.zeros(20, dtype=np.complex128)
    with pytest.raises(ValueError):
        oracle.frames(x, 8, 0, 2)
    with pytest.raises(ValueError):
        oracle.frames(x, 8, 7, 3)          # needs 2*7 + 8 = 22 samples
    with pytest.raises(ValueError):
        oracle.frames(x, 8, 4, 2, np.ones(7))
    assert oracle.frames(x, 8, 6, 3).shape == (3, 8)


# --- real-input segments -----------------------------------------------------

@pytest.mark.parametrize("n", [2, 8, 1000, 1024])
def test_real_forward_matches_numpy_rfft(n):
    x = np.random.default_rng(n).standard_normal((5, n))
    assert np.allclose(oracle.real_forward(x, n), np.fft.rfft(x, axis=1),
                       rtol=1e-12, atol=1e-9 * n)
    x32 = x.astype(np.float32)
    assert np.allclose(oracle.real_inverse(oracle.real_forward(x32, n), n),
                       n * x32.astype(np.float64), atol=1e-9 * n)


@pytest.mark.parametrize("n,k0", [(64, 5), (1000, 499), (16, 8), (16, 0)])
def test_real_cosine_closed_form(n, k0):
    """cos(2 pi k0 j / n) has n/2 at bin k0 (n at k0 = 0 or n/2) and zeros
    elsewhere among bins 0..n/2."""
    j = np.arange(n)
    y = oracle.real_forward(np.cos(2 * np.pi * k0 * j / n), n)[0]
    want = np.zeros(n // 2 + 1)
    want[k0] = n if k0 in (0, n // 2) else n / 2
    assert np.max(np.abs(y - want)) < 1e-9 * n


def test_real_inverse_definition_and_edge_bins():
    n = 12
    rng = np.random.default_rng(9)
    h = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    x = oracle.real_inverse(h, n)[0]
    # direct sum over the Hermitian extension, real bins 0 and n/2
    full = np.concatenate([h, np.conj(h[1:6][::-1])])
    full[0], full[6] = full[0].real, full[6].real
    for jj in range(n):
        s = sum(full[k] * np.exp(2j * np.pi * jj * k / n) for k in range(n))
        assert abs(s.imag) < 1e-9 and abs(s.real - x[jj]) < 1e-9
    # imaginary parts of bins 0 and n/2 do not matter
    h2 = h.copy()
    h2[0] += 3j
    h2[6] -= 2j
    assert np.allclose(oracle.real_inverse(h2, n), x, atol=1e-12)
    assert np.allclose(x, np.fft.irfft(h, n) * n, atol=1e-9)


def test_real_bad_arguments():
    with pytest.raises(ValueError):
        oracle.real_forward(np.zeros(9), 9)
    with pytest.raises(TypeError):
        oracle.real_forward(np.zeros(8, dtype=np.complex64), 8)
    with pytest.raises(ValueError):
        oracle.real_inverse(np.zeros(6, dtype=np.complex128), 8)
