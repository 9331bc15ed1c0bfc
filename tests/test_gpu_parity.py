"""GPU parity: the HIP path against the FP64 oracle, element by element,
per-segment relative L2 error <= 5e-7 * log2(N)."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
from siggen import workloads

from gpu_helpers import announce, check, noise, run

pytestmark = pytest.mark.gpu

SINGLE = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1000, 1024, 1536, 2048, 4096,
          6000, 8192, 16384]
FOUR_STEP = [1 << 15, 1 << 16, 1 << 17, 1 << 18, 1 << 20]
FALLBACK = [3, 5, 6, 9, 12, 15, 25, 27, 30, 45, 81, 100, 125, 243, 360,
            3 ** 9, 5 ** 6, 2 * 3 ** 9]


def ragged_batch(n):
    """A batch spanning several workgroups with a ragged tail."""
    if n <= 64:
        return 200 + 7
    if n <= 4096:
        return max(3, (1 << 18) // n) + 3
    return 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fs.lib()
    yield


def test_small_workload_all_segments():
    n, b = 1024, 1024
    announce("1024-point x 1024 segments, all vs recursive oracle, 64 vs direct")
    x = workloads.small_signal().segments(0, b)
    y = run(n, x)
    check(n, y, x, what="all segments")
    idx = np.random.default_rng(0).choice(b, 64, replace=False)
    ref = oracle.dft_direct(x[idx], n)
    assert np.all(oracle.rel_l2(y[idx], ref) <= oracle.tolerance(n))
    # the three unit tones (phase 0) give N at their bins in every segment,
    # plus the noise's share of that bin (complex std sqrt(2N) = 45): their
    # mean over the 1024 segments is N within 2 % (about 14 standard
    # deviations of that mean), and the other bins average near 0
    tone_bins = [b0 for b0, _, _ in workloads.small_signal().tones]
    mean = y.astype(np.complex128).mean(axis=0)
    for b0 in tone_bins:
        assert abs(mean[b0] - n) < 0.02 * n, (b0, mean[b0])
    others = np.delete(np.abs(mean), tone_bins)
    assert others.max() < 0.02 * n


@pytest.mark.parametrize("n", SINGLE + FOUR_STEP + FALLBACK)
@pytest.mark.parametrize("direction", [fs.FORWARD, fs.INVERSE])
def test_lengths(n, direction):
    b = ragged_batch(n)
    announce("n=%d batch=%d dir=%d" % (n, b, direction))
    x = noise(n, b, seed=n)
    check(n, run(n, x, direction), x, direction)


@pytest.mark.parametrize("n", [256, 512, 1000, 1024, 1536, 2048, 4096, 6000, 8192, 16384])
def test_every_variant(n):
    for v in range(fs.variant_count(n)):
        b = ragged_batch(n)
        announce("n=%d variant=%d batch=%d" % (n, v, b))
        x = noise(n, b, seed=10 * n + v)
        for d in (fs.FORWARD, fs.INVERSE):
            check(n, run(n, x, d, variant=v), x, d, what="variant %d dir %d" % (v, d))


@pytest.mark.parametrize("n", [4096, 8192, 16384])
def test_every_variant_walks_several_segments(n, monkeypatch):
    """A persistent grid of one resident wave of workgroups, so every
    workgroup transforms several segments in turn and reuses its LDS (the
    batches above fit one segment per workgroup at these lengths)."""
    monkeypatch.setenv("FFTSEG_GRID_MULT", "1")
    b = (1 << 24) // n + 5
    x = noise(n, b, seed=n + 3)
    ref = {d: oracle.fft_recursive(x, n, d) for d in (fs.FORWARD, fs.INVERSE)}
    for v in range(fs.variant_count(n)):
        announce("n=%d variant=%d batch=%d grid_mult=1" % (n, v, b))
        for d in (fs.FORWARD, fs.INVERSE):
            e = oracle.rel_l2(run(n, x, d, variant=v), ref[d])
            assert np.all(e <= oracle.tolerance(n)), (v, d, float(e.max()))


@pytest.mark.parametrize("n,b", [(1 << 15, 400), (1 << 16, 200), (1 << 18, 40), (1 << 20, 9),
                                 (1 << 22, 3)])
def test_four_step_tiles_walk_several_tiles(monkeypatch, n, b):
    """The same for the column and row passes of two-pass splits: every
    column and every row tile variant, at batches that give each resident
    workgroup two or more tiles (tiles alternate LDS twiddle buffers)."""
    import torch
    monkeypatch.setenv("FFTSEG_GRID_MULT", "1")
    n1, n2, nc, nr = fs.split_info(n)
    x = noise(n, b, seed=29)
    ref = {d: oracle.fft_recursive(x, n, d) for d in (fs.FORWARD, fs.INVERSE)}
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    for c, r in [(min(v, nc - 1), min(v, nr - 1)) for v in range(max(nc, nr))]:
        announce("n=%d column variant %d row variant %d batch=%d grid_mult=1" % (n, c, r, b))
        for d in (fs.FORWARD, fs.INVERSE):
            with fs.Plan(n, b, d, split_variants=(c, r)) as p:
                if (c, r) == (0, 0):
                    # the default tiles below 1024 points keep Y in 16-column blocks
                    assert p.describe()["y_blocked"] == int(n1 < 1024 and n2 < 1024)
                y = p.exec(xd).cpu().numpy().reshape(b, n)
            e = oracle.rel_l2(y, ref[d])
            assert np.all(e <= oracle.tolerance(n)), (c, r, d, float(e.max()))


@pytest.mark.parametrize("n", [1 << 15, 1 << 16, 1 << 18, 1 << 20, 1 << 22])
def test_every_four_step_tile_variant(n):
    n1, n2, nc, nr = fs.split_info(n)
    assert n1 * n2 == n and nc >= 1 and nr >= 1
    b = 3 if n < 1 << 20 else 2
    x = noise(n, b, seed=n + 17)
    ref = {d: oracle.fft_recursive(x, n, d) for d in (fs.FORWARD, fs.INVERSE)}
    for c in range(nc):
        for r in range(nr):
            announce("n=%d split %dx%d column variant %d row variant %d" % (n, n1, n2, c, r))
            for d in (fs.FORWARD, fs.INVERSE):
                import torch
                xd = torch.from_numpy(x.reshape(-1)).cuda()
                with fs.Plan(n, b, d, split_variants=(c, r)) as p:
                    y = p.exec(xd).cpu().numpy().reshape(b, n)
                e = oracle.rel_l2(y, ref[d])
                assert np.all(e <= oracle.tolerance(n)), (c, r, d, e.max())


@pytest.mark.parametrize("n", [1000, 4096, 1 << 15, 1 << 16, 1 << 18, 1 << 20, 1 << 22])
def test_bases_off_a_line_boundary(n):
    """Input and output base pointers anywhere in a 128-byte line (two-pass
    plans then start their blocks mid-segment and wrap round), out of place
    and in place; nothing outside the output range is written."""
    import torch
    b = 3 if n <= 1 << 18 else 2
    x = noise(n, b, seed=n + 9).reshape(-1)
    ref = oracle.fft_recursive(x.reshape(b, n), n)
    for lead_in, lead_out in [(8, 8), (3, 5), (0, 13), (15, 0)]:
        announce("n=%d batch=%d lead in %d out %d" % (n, b, lead_in, lead_out))
        xd = torch.zeros(b * n + 16, dtype=torch.complex64, device="cuda")
        xd[lead_in:lead_in + b * n] = torch.from_numpy(x).cuda()
        yd = torch.zeros(b * n + 16, dtype=torch.complex64, device="cuda")
        with fs.Plan(n, b) as p:
            p.exec_ptr(xd.data_ptr() + 8 * lead_in, yd.data_ptr() + 8 * lead_out, 0)
            torch.cuda.synchronize()
            y = yd.cpu().numpy()
            assert np.all(y[:lead_out] == 0) and np.all(y[lead_out + b * n:] == 0)
            got = y[lead_out:lead_out + b * n].reshape(b, n)
            assert np.all(oracle.rel_l2(got, ref) <= oracle.tolerance(n)), (lead_in, lead_out)
            # in place at the input's offset
            p.exec_ptr(xd.data_ptr() + 8 * lead_in, xd.data_ptr() + 8 * lead_in, 0)
            torch.cuda.synchronize()
            got2 = xd.cpu().numpy()[lead_in:lead_in + b * n].reshape(b, n)
            assert np.array_equal(got2, y[lead_out:lead_out + b * n].reshape(b, n)) or \
                np.all(oracle.rel_l2(got2, ref) <= oracle.tolerance(n))


def test_shifted_tiles_walk_several_tiles(monkeypatch):
    """The line-aligned (shifted, wrapping) four-step tiles and the rotated
    one-pass kernel on a persistent grid of one resident wave, so every
    workgroup takes several tiles or segments in turn."""
    import torch
    monkeypatch.setenv("FFTSEG_GRID_MULT", "1")
    for n, b in [(1 << 16, 300), (4096, 4101)]:
        x = noise(n, b, seed=n + 21).reshape(-1)
        ref = oracle.fft_recursive(x.reshape(b, n), n)
        announce("n=%d batch=%d lead in 5 out 3, grid_mult=1" % (n, b))
        xd = torch.zeros(b * n + 16, dtype=torch.complex64, device="cuda")
        xd[5:5 + b * n] = torch.from_numpy(x).cuda()
        yd = torch.zeros(b * n + 16, dtype=torch.complex64, device="cuda")
        with fs.Plan(n, b) as p:
            p.exec_ptr(xd.data_ptr() + 40, yd.data_ptr() + 24, 0)
        torch.cuda.synchronize()
        got = yd.cpu().numpy()[3:3 + b * n].reshape(b, n)
        assert np.all(oracle.rel_l2(got, ref) <= oracle.tolerance(n))


@pytest.mark.parametrize("n", [1 << 21, 3 * (1 << 20), 1 << 23, 1 << 24])
def test_long_lengths_up_to_the_cap(n):
    """Segments up to the 2^24-sample cap (two passes where both halves
    have tiles, the radix-stage path otherwise), both directions."""
    b = 2 if n <= 1 << 21 else 1
    announce("n=%d batch=%d (%s)" % (n, b, fs.Plan(n, b).describe()["kind"]))
    x = noise(n, b, seed=n + 5)
    for d in (fs.FORWARD, fs.INVERSE):
        check(n, run(n, x, d), x, d, what="long dir %d" % d)


@pytest.mark.parametrize("n", [1024, 4096, 6000, 1 << 16, 3 ** 9, 5])
def test_in_place_equals_out_of_place_and_deterministic(n):
    b = ragged_batch(n)
    announce("in place n=%d" % n)
    x = noise(n, b, seed=7)
    a = run(n, x)
    assert np.array_equal(a, run(n, x, inplace=True))
    assert np.array_equal(a, run(n, x))


@pytest.mark.parametrize("n", [1024, 1536, 1 << 16])
def test_segment_locality_and_order(n):
    b = 9
    announce("locality n=%d" % n)
    x = noise(n, b, seed=3)
    y = run(n, x)
    x2 = x.copy()
    x2[4] += noise(n, 1, seed=4)[0]
    y2 = run(n, x2)
    assert np.array_equal(np.delete(y, 4, 0), np.delete(y2, 4, 0))
    assert not np.array_equal(y[4], y2[4])
    perm = np.random.default_rng(1).permutation(b)
    assert np.array_equal(run(n, x[perm]), y[perm])


@pytest.mark.parametrize("n", [1000, 4096, 1 << 20])
def test_round_trip(n):
    b = 2 if n > 4096 else 33
    announce("round trip n=%d" % n)
    x = noise(n, b, seed=11)
    z = run(n, run(n, x), fs.INVERSE) / n
    err = oracle.rel_l2(z, x.astype(np.complex128))
    assert np.all(err <= 2 * oracle.tolerance(n)), err.max()


def test_closed_forms():
    announce("closed forms")
    n = 4096
    x = np.zeros((3, n), np.complex64)
    x[0, 0] = 1                     # impulse: flat spectrum
    x[1, 5] = 1                     # shifted impulse: phase ramp
    k0 = 1234
    t = np.arange(n)
    x[2] = np.exp(2j * np.pi * ((k0 * t) % n) / n)   # bin tone: one spike
    y = run(n, x).astype(np.complex128)
    assert np.allclose(y[0], 1, atol=1e-6)
    k = np.arange(n)
    assert np.allclose(y[1], np.exp(-2j * np.pi * ((5 * k) % n) / n), atol=1e-6)
    spike = np.zeros(n)
    spike[k0] = n
    assert np.abs(y[2] - spike).max() < 1e-6 * n
    # unit chirp exp(i pi t^2/N): X[k] = sqrt(N) e^{i pi/4} e^{-i pi k^2/N}
    n = 1 << 20
    t = np.arange(n, dtype=np.int64)
    c = np.exp(1j * np.pi * ((t * t) % (2 * n)) / n).astype(np.complex64)
    want = np.sqrt(n) * np.exp(1j * np.pi / 4) * np.exp(-1j * np.pi * ((t * t) % (2 * n)) / n)
    yc = run(n, c[None, :])[0]
    assert oracle.rel_l2(yc[None], want[None])[0] <= oracle.tolerance(n)


def test_length_one_is_identity():
    announce("n=1")
    x = noise(1, 10, seed=5)
    assert np.array_equal(run(1, x), x)
    assert np.array_equal(run(1, x, fs.INVERSE), x)
    # the copy kernel's cases: 16-byte accesses (even count, aligned), 8-byte
    # accesses (odd count, or a pointer off a 16-byte boundary), several
    # workgroup tiles with a ragged last one
    import torch
    for b, lead in [(2 * 2048 * 3 + 2, 0), (2048 * 5 + 3, 0), (4096 * 2 + 6, 1)]:
        x = noise(1, b + lead, seed=b).reshape(-1)
        xd = torch.from_numpy(x).cuda()
        yd = torch.zeros(b + 1, dtype=torch.complex64, device="cuda")
        with fs.Plan(1, b) as p:
            p.exec_ptr(xd.data_ptr() + 8 * lead, yd.data_ptr() + 8 * lead, 0)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        assert np.array_equal(y[lead:lead + b], x[lead:lead + b])
        assert np.all(y[:lead] == 0) and np.all(y[lead + b:] == 0)


def test_zero_input_gives_exact_zero():
    announce("zeros")
    for n in (4096, 1 << 16, 3 ** 9):
        x = np.zeros((2, n), np.complex64)
        assert not np.any(run(n, x))


# ----- argument checks with a live device ---------------------------------

def _hip():
    return ctypes.CDLL("libamdhip64.so")


def test_exec_argument_errors():
    import torch
    announce("exec argument errors")
    n, b = 1024, 4
    x = torch.zeros(n * b + 8, dtype=torch.complex64, device="cuda")
    p = fs.Plan(n, b)
    base = x.data_ptr()
    with pytest.raises(fs.FFTError) as e:
        p.exec_ptr(base, base + 8 * 8)              # partial overlap
    assert e.value.name == "FFT_ERR_OVERLAP"
    with pytest.raises(fs.FFTError) as e:
        p.exec_ptr(base + 4, base + 4)              # misaligned
    assert e.value.name == "FFT_ERR_ALIGNMENT"
    with pytest.raises(fs.FFTError) as e:
        p.exec_ptr(base, 0)
    assert e.value.name == "FFT_ERR_INVALID_ARG"
    with pytest.raises(fs.FFTError) as e:
        p.exec_ptr(base, base, batch=b + 1)
    assert e.value.name == "FFT_ERR_INVALID_ARG"
    p.exec_ptr(base, base, batch=b - 1)             # a prefix is fine
    torch.cuda.synchronize()
    p.close()


def test_exec_rejects_memory_it_cannot_use():
    """Buffers the library must refuse: too short for the batch, or
    ordinary host memory.  Each case runs only after checking, with the HIP
    runtime directly, that the runtime reports the buffer the way the
    library's check relies on, so no kernel can run on a bad pointer."""
    import torch
    announce("exec bounds / host pointer")
    hip = _hip()
    torch.cuda.synchronize()
    p = ctypes.c_void_p()
    nbytes = 1 << 20
    assert hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes)) == 0
    try:
        base, size = ctypes.c_void_p(), ctypes.c_size_t()
        rc = hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), p)
        if rc == 0 and base.value == p.value and size.value == nbytes:
            plan = fs.Plan(1024, 2 * nbytes // 8 // 1024)   # needs 2 MiB
            with pytest.raises(fs.FFTError) as e:
                plan.exec_ptr(p.value, p.value)
            assert e.value.name == "FFT_ERR_BOUNDS"
            plan.close()
    finally:
        hip.hipFree(p)
    host = np.zeros(1024 * 2, np.complex64)
    hp = ctypes.c_void_p(host.ctypes.data)
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    attr = (ctypes.c_int * 32)()
    range_rc = hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), hp)
    attr_rc = hip.hipPointerGetAttributes(attr, hp)
    hip.hipGetLastError()
    # hipMemoryTypeDevice = 2, hipMemoryTypeManaged = 3
    if range_rc != 0 and (attr_rc != 0 or attr[0] not in (2, 3)):
        plan = fs.Plan(1024, 2)
        with pytest.raises(fs.FFTError) as e:
            plan.exec_ptr(host.ctypes.data, host.ctypes.data)
        assert e.value.name == "FFT_ERR_INVALID_ARG"
        plan.close()


def test_plan_describe():
    announce("describe")
    d = fs.Plan(4096, 8).describe()
    assert d["kind"] == "single_pass" and d["radices"] == fs.factorize(4096)
    assert int(np.prod(d["radices"])) == 4096
    d = fs.Plan(1 << 20, 2).describe()
    assert d["kind"] == "four_step" and d["n1"] * d["n2"] == 1 << 20
    d = fs.Plan(3 ** 9, 2).describe()
    assert d["kind"] == "radix_stages"


def test_small_batches_take_the_small_batch_kernel():
    """A batch that gives a length's default kernel fewer than two
    workgroups per CU takes the length's small-batch kernel, unless a
    variant is forced; both agree with the oracle."""
    import torch
    announce("small-batch kernels")
    for n, small, large, small_variant in [(1024, 1024, 1 << 16, 7), (2048, 256, 1 << 14, 6)]:
        with fs.Plan(n, small) as p:
            assert p.describe()["variant"] == small_variant
        with fs.Plan(n, large) as p:
            assert p.describe()["variant"] == 0
        with fs.Plan(n, small, fs.FORWARD, 0) as p:
            assert p.describe()["variant"] == 0
        x = noise(n, small, seed=n + 5)
        ref = oracle.fft_recursive(x, n)
        with fs.Plan(n, small) as p:
            y = p.exec(torch.from_numpy(x.reshape(-1)).cuda()).cpu().numpy().reshape(small, n)
        assert np.all(oracle.rel_l2(y, ref) <= oracle.tolerance(n))


@pytest.mark.parametrize("n,b,sub", [(1 << 16, 7, 2), (1 << 18, 5, 2), (1 << 20, 5, 2)])
@pytest.mark.parametrize("lead", [0, 3])
def test_two_pass_plans_across_sub_batches(monkeypatch, n, b, sub, lead):
    """Two-pass plans whose batch runs as several sub-batches through the
    one scratch buffer (a ragged last one), with Y in 16-column blocks where
    the plan's tiles have that form, from bases on a line and `lead` samples
    past one."""
    import torch
    monkeypatch.setenv("FFTSEG_SUB_SAMPLES", str(sub * n))
    x = noise(n, b, seed=n + 41)
    for d in (fs.FORWARD, fs.INVERSE):
        announce("n=%d batch=%d sub-batch=%d lead=%d dir=%d" % (n, b, sub, lead, d))
        xd = torch.zeros(n * b + 16, dtype=torch.complex64, device="cuda")
        xd[lead:lead + n * b] = torch.from_numpy(x.reshape(-1))
        yd = torch.zeros_like(xd)
        with fs.Plan(n, b, d) as p:
            desc = p.describe()
            assert desc["sub_batch"] == sub
            p.exec(xd[lead:lead + n * b], yd[lead:lead + n * b])
        y = yd.cpu().numpy()
        assert not y[:lead].any() and not y[lead + n * b:].any()
        check(n, y[lead:lead + n * b].reshape(b, n), x, d,
              what="y_blocked %d" % desc["y_blocked"])
