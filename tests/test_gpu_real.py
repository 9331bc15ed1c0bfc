"""Real-input segments (fft_plan_create_real) against the FP64 oracle:
forward bins 0..N/2 of float32 segments, inverse back to float32 samples,
every length with a fused real kernel and lengths whose half runs as a
two-pass or radix-stage plan with a separate split pass, ragged batches,
argument errors."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
import siggen

from gpu_helpers import announce

pytestmark = pytest.mark.gpu

REAL_LENGTHS = [4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768,
                2000, 3072, 12000]
# N/2 without a one-pass kernel: four-step (65536, 2^17, 2^21) or radix
# stages (2 * 3^9, 2 * 5^6)
SPLIT_LENGTHS = [1 << 16, 1 << 17, 1 << 21, 2 * 3 ** 9, 2 * 5 ** 6]


def real_samples(n, batch, seed):
    # real and imaginary parts of the seeded complex noise, as 2*n*batch/2 reals
    z = siggen.Signal(seed=seed, seg_len=n, sigma=1.0).samples(0, n * batch // 2 + 1)
    return z.view(np.float32)[: n * batch].copy()


def run_real(n, batch, x, direction):
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    with fs.RealPlan(n, batch, direction) as p:
        y = p.exec(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("n", REAL_LENGTHS + SPLIT_LENGTHS)
def test_real_forward_and_inverse(n):
    batch = max(3, min(257, (1 << 21) // n)) | 1          # odd: ragged last tile
    announce("real n=%d batch=%d" % (n, batch))
    x = real_samples(n, batch, 50 + n % 97)
    got = run_real(n, batch, x, fs.FORWARD).reshape(batch, n // 2 + 1)
    ref = oracle.real_forward(x, n)
    err = oracle.rel_l2(got, ref)
    print("  forward max rel-L2 %.3e" % err.max(), flush=True)
    assert np.all(err <= oracle.tolerance(n)), err.max()
    # inverse of the oracle's spectrum (rounded to complex64) back to reals
    spec = ref.astype(np.complex64)
    back = run_real(n, batch, spec.reshape(-1), fs.INVERSE).reshape(batch, n)
    want = oracle.real_inverse(spec, n)
    e2 = np.linalg.norm(back - want, axis=1) / np.linalg.norm(want, axis=1)
    print("  inverse max rel-L2 %.3e" % e2.max(), flush=True)
    assert np.all(e2 <= oracle.tolerance(n)), e2.max()


def test_real_inverse_ignores_edge_imaginary_parts():
    n, batch = 1024, 5
    announce("real inverse edge bins")
    rng = np.random.default_rng(7)
    spec = (rng.standard_normal((batch, n // 2 + 1)) +
            1j * rng.standard_normal((batch, n // 2 + 1))).astype(np.complex64)
    got = run_real(n, batch, spec.reshape(-1), fs.INVERSE).reshape(batch, n)
    want = oracle.real_inverse(spec, n)
    e = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
    assert np.all(e <= oracle.tolerance(n)), e.max()


def test_real_cosine_bins():
    n, batch = 4096, 4
    announce("real cosine bins")
    j = np.arange(n)
    x = np.stack([np.cos(2 * np.pi * k0 * j / n) for k0 in (0, 1, 777, n // 2)])
    got = run_real(n, batch, x.astype(np.float32).reshape(-1), fs.FORWARD).reshape(batch, -1)
    ref = oracle.real_forward(x.astype(np.float32), n)
    assert np.all(oracle.rel_l2(got, ref) <= oracle.tolerance(n))
    for s, k0 in enumerate((0, 1, 777, n // 2)):
        assert abs(got[s, k0] - ref[s, k0]) < 1e-3 * n


def test_real_plan_errors():
    import torch
    announce("real plan errors")
    for n in (7, 2, 2 * 7 * 64, 1 << 25):
        with pytest.raises(fs.FFTError) as e:
            fs.RealPlan(n, 4)
        assert e.value.name == "FFT_ERR_UNSUPPORTED_LENGTH", n
    n, b = 1024, 4
    x = torch.zeros(n * b, dtype=torch.float32, device="cuda")
    big = torch.zeros((n // 2 + 1) * b * 2, dtype=torch.complex64, device="cuda")
    with fs.RealPlan(n, b) as p:
        with pytest.raises(fs.FFTError) as e:          # in place
            p.exec_ptr(big.data_ptr(), big.data_ptr())
        assert e.value.name == "FFT_ERR_OVERLAP"
        with pytest.raises(fs.FFTError) as e:          # complex-only entry point
            p.exec_frames_ptr(x.data_ptr(), x.numel(), big.data_ptr(), 2, 512)
        assert e.value.name == "FFT_ERR_INVALID_ARG"
        with pytest.raises(fs.FFTError) as e:
            p.exec_graph_ptr(x.data_ptr(), big.data_ptr())
        assert e.value.name == "FFT_ERR_INVALID_ARG"
        assert p.describe()["kind"] == "real"
    torch.cuda.synchronize()
    # an output allocation one byte short of the batch's bins
    hip = ctypes.CDLL("libamdhip64.so")
    q = ctypes.c_void_p()
    nbytes = (n // 2 + 1) * b * 8 - 8
    assert hip.hipMalloc(ctypes.byref(q), ctypes.c_size_t(nbytes)) == 0
    try:
        base, size = ctypes.c_void_p(), ctypes.c_size_t()
        rc = hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), q)
        if rc == 0 and base.value == q.value and size.value == nbytes:
            with fs.RealPlan(n, b) as p:
                with pytest.raises(fs.FFTError) as e:
                    p.exec_ptr(x.data_ptr(), q.value)
                assert e.value.name == "FFT_ERR_BOUNDS"
    finally:
        hip.hipFree(q)


def test_real_separate_split_over_sub_batches():
    """A separate-split plan whose batch spans two sub-batches (2^28 complex
    values of the half length each): rows repeat with period 2, so the rows
    of the second sub-batch must equal those of the first bit for bit, and
    the first two match the oracle."""
    import torch
    n, batch = 1 << 21, 258
    announce("real separate split n=%d batch=%d" % (n, batch))
    with fs.RealPlan(n, batch) as p:
        d = p.describe()
        assert d["kind"] == "real" and d["separate_split"] == 1 and d["sub_batch"] == 256
    x2 = real_samples(n, 2, 77)
    xd = torch.from_numpy(x2).to("cuda").repeat(batch // 2)
    with fs.RealPlan(n, batch, fs.FORWARD) as p:
        y = p.exec(xd).reshape(batch, n // 2 + 1)
    torch.cuda.synchronize()
    assert torch.equal(y[256:258], y[0:2])
    ref = oracle.real_forward(x2, n)
    assert np.all(oracle.rel_l2(y[0:2].cpu().numpy(), ref) <= oracle.tolerance(n))
    spec = torch.from_numpy(ref.astype(np.complex64).reshape(-1)).to("cuda").repeat(batch // 2)
    with fs.RealPlan(n, batch, fs.INVERSE) as p:
        back = p.exec(spec).reshape(batch, n)
    torch.cuda.synchronize()
    assert torch.equal(back[256:258], back[0:2])
    want = oracle.real_inverse(ref.astype(np.complex64), n)
    b2 = back[0:2].cpu().numpy()
    e = np.linalg.norm(b2 - want, axis=1) / np.linalg.norm(want, axis=1)
    assert np.all(e <= oracle.tolerance(n)), e.max()
