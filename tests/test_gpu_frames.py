"""Overlapping, windowed segments (fft_exec_frames) against the FP64
oracle's short-time transform, on every plan kind: one-pass lengths read
the frames in the kernel, two-pass lengths in their column pass, radix-stage
lengths gather first."""
import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
import siggen

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def hann32(n):
    j = np.arange(n, dtype=np.float64)
    return (0.5 - 0.5 * np.cos(2 * np.pi * j / n)).astype(np.float32)


def run_frames(n, x, hop, n_frames, window, direction=fs.FORWARD, batch=None):
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")
    wd = None if window is None else torch.from_numpy(window).to("cuda")
    with fs.Plan(n, batch or n_frames, direction) as p:
        y = p.exec_frames(xd, hop, n_frames, wd)
    torch.cuda.synchronize()
    return y.cpu().numpy().reshape(n_frames, n)


@pytest.mark.parametrize("n,hop,frames", [
    (1024, 256, 37),        # 75 % overlap, ragged last tile
    (4096, 1024, 21),
    (4096, 4096, 9),        # disjoint
    (4096, 4099, 5),        # gaps between frames
    (1000, 333, 17),        # non power of two, odd hop
    (16384, 8192, 7),
    (8192, 2048, 9),        # the length's frame kernel is not its default's
    (2048, 512, 11),
    (1 << 16, 1 << 14, 5),  # two-pass lengths: read by the column pass
    (1 << 15, 1000, 6),
    (1 << 18, 70001, 4),
    (1 << 20, 1 << 18, 3),  # the 1024-point column tiles' frame form
    (3 ** 9, 5000, 4),      # radix-stage fallback
    (1, 1, 11),             # identity length
])
@pytest.mark.parametrize("windowed", [True, False])
def test_frames_match_oracle(n, hop, frames, windowed):
    announce("frames n=%d hop=%d frames=%d window=%s" % (n, hop, frames, windowed))
    total = (frames - 1) * hop + n + 7          # a few samples past the last frame
    x = siggen.Signal(seed=41, seg_len=1, sigma=1.0).samples(0, total)
    w = hann32(n) if windowed else None
    got = run_frames(n, x, hop, frames, w)
    ref = oracle.short_time(x, n, hop, frames, w)
    err = oracle.rel_l2(got, ref)
    print("  max rel-L2 %.3e" % err.max(), flush=True)
    assert np.all(err <= oracle.tolerance(n)), err.max()


def test_frames_with_every_4096_variant():
    """A plan forced to a kernel variant uses that variant's frame form when
    it has one and the length's default frame kernel otherwise: all agree
    with the oracle."""
    n, hop, frames = 4096, 1536, 19
    x = siggen.Signal(seed=44, seg_len=1, sigma=1.0).samples(0, (frames - 1) * hop + n)
    w = hann32(n)
    ref = oracle.short_time(x, n, hop, frames, w)
    import torch
    xd = torch.from_numpy(x).to("cuda")
    wd = torch.from_numpy(w).to("cuda")
    for v in range(fs.variant_count(n)):
        announce("frames n=%d variant %d" % (n, v))
        with fs.Plan(n, frames, fs.FORWARD, v) as p:
            y = p.exec_frames(xd, hop, frames, wd).cpu().numpy().reshape(frames, n)
        assert np.all(oracle.rel_l2(y, ref) <= oracle.tolerance(n)), v


def test_frames_inverse_and_smaller_than_plan():
    n, hop, frames = 2048, 512, 13
    announce("frames inverse n=%d" % n)
    x = siggen.Signal(seed=42, seg_len=1, sigma=1.0).samples(0, (frames - 1) * hop + n)
    w = np.random.default_rng(3).uniform(0.0, 1.0, n).astype(np.float32)
    got = run_frames(n, x, hop, frames, w, fs.INVERSE, batch=64)
    ref = oracle.short_time(x, n, hop, frames, w, fs.INVERSE)
    assert np.all(oracle.rel_l2(got, ref) <= oracle.tolerance(n))


def test_frames_hop_n_equals_segments():
    """hop == n without a window is the plain disjoint transform: both
    within the bar of the oracle's records (the two run different kernel
    instances, so their roundings may differ)."""
    n, b = 4096, 24
    announce("frames hop=n vs exec")
    import torch
    x = siggen.Signal(seed=43, seg_len=n, sigma=1.0).samples(0, n * b)
    xd = torch.from_numpy(x).to("cuda")
    with fs.Plan(n, b) as p:
        a = p.exec(xd).cpu().numpy().reshape(b, n)
        f = p.exec_frames(xd, n).cpu().numpy().reshape(b, n)
    ref = oracle.fft_recursive(x, n)
    assert np.all(oracle.rel_l2(a, ref) <= oracle.tolerance(n))
    assert np.all(oracle.rel_l2(f, ref) <= oracle.tolerance(n))
    assert np.all(oracle.rel_l2(f, a) <= 2 * oracle.tolerance(n))


def test_frames_argument_errors():
    import torch
    n = 1024
    announce("frames argument errors")
    x = torch.zeros(n * 8, dtype=torch.complex64, device="cuda")
    out = torch.empty(n * 8, dtype=torch.complex64, device="cuda")
    with fs.Plan(n, 8) as p:
        cases = [
            (lambda: p.exec_frames_ptr(x.data_ptr(), x.numel(), out.data_ptr(), 8, 1024 + 1),
             "FFT_ERR_BOUNDS"),
            (lambda: p.exec_frames_ptr(x.data_ptr(), x.numel(), out.data_ptr(), 9, 512),
             "FFT_ERR_INVALID_ARG"),
            (lambda: p.exec_frames_ptr(x.data_ptr(), x.numel(), out.data_ptr(), 2, 0),
             "FFT_ERR_INVALID_ARG"),
            (lambda: p.exec_frames_ptr(x.data_ptr(), x.numel(), x.data_ptr() + 8 * 64, 2, 64),
             "FFT_ERR_OVERLAP"),
            (lambda: p.exec_frames_ptr(x.data_ptr() + 4, n * 2, out.data_ptr(), 2, 64),
             "FFT_ERR_ALIGNMENT"),
        ]
        for f, name in cases:
            with pytest.raises(fs.FFTError) as e:
                f()
            assert e.value.name == name
    torch.cuda.synchronize()


def test_two_pass_frames_across_sub_batches():
    """2^20-point frames, more of them than one scratch sub-batch holds
    (512): frames on both sides of the boundary against the oracle."""
    import torch
    n, hop, frames = 1 << 20, 4099, 513
    announce("frames n=%d hop=%d frames=%d" % (n, hop, frames))
    total = (frames - 1) * hop + n
    x = siggen.Signal(seed=45, seg_len=1, sigma=1.0).samples(0, total)
    w = hann32(n)
    xd = torch.from_numpy(x).to("cuda")
    wd = torch.from_numpy(w).to("cuda")
    with fs.Plan(n, frames) as p:
        assert p.describe()["sub_batch"] == 512
        y = p.exec_frames(xd, hop, frames, wd)
    torch.cuda.synchronize()
    for f in (0, 1, 511, 512):
        got = y[f * n:(f + 1) * n].cpu().numpy()[None]
        ref = oracle.short_time(x[f * hop:f * hop + n], n, hop, 1, w)
        assert oracle.rel_l2(got, ref)[0] <= oracle.tolerance(n), f


@pytest.mark.parametrize("n,hop,frames,variant", [
    (4096, 1024, 1601, 3),     # the length's frame kernel (cached overlapping loads)
    (4096, 1024, 1601, 15),    # frames dealt to the XCDs in contiguous runs
    (4096, 4096, 901, 3),      # disjoint frames: streamed loads
    (8192, 2048, 701, 7),
    (16384, 4096, 701, 0),     # split exchanges
    (4096, 1024, 1601, None),  # default plans: the frame kernel of another row
    (8192, 2048, 701, None),
])
def test_frame_kernels_walk_several_groups(monkeypatch, n, hop, frames, variant):
    """Frame kernels on a persistent grid of one resident wave of workgroups:
    each workgroup takes several frame groups and the last sweep is ragged."""
    import torch
    monkeypatch.setenv("FFTSEG_GRID_MULT", "1")
    announce("frames walk n=%d hop=%d frames=%d variant=%s" % (n, hop, frames, variant))
    x = siggen.Signal(seed=47, seg_len=1, sigma=1.0).samples(0, (frames - 1) * hop + n)
    w = hann32(n)
    xd = torch.from_numpy(x).to("cuda")
    wd = torch.from_numpy(w).to("cuda")
    with fs.Plan(n, frames, fs.FORWARD, variant) as p:
        assert p.describe()["grid_mult"] == 1
        y = p.exec_frames(xd, hop, frames, wd).cpu().numpy().reshape(frames, n)
    err = oracle.rel_l2(y, oracle.short_time(x, n, hop, frames, w))
    assert np.all(err <= oracle.tolerance(n)), float(err.max())
