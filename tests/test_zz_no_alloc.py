"""fft_exec_segments_noalloc (no plan, no device allocation: tables and
the two-pass Y buffer live in the library's static device array) against
fft_exec_segments of a plan on the same input, through the C ABI: two calls
in a row per length, the second with a smaller batch, then the oracle on a
sample."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs

from gpu_helpers import announce, noise

pytestmark = pytest.mark.gpu


def _noalloc(n, batch, direction, xp, yp, stream):
    """The C entry point itself (its ctypes prototype set here)."""
    f = ctypes.CDLL(fs.LIB_PATH).fft_exec_segments_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    rc = f(n, batch, direction, xp, yp, stream)
    if rc != 0:
        raise fs.FFTError(rc, fs.last_error())


# one-pass lengths (tables only), two-pass lengths with several sub-batches
# of the static Y buffer (2^24 samples: 16 segments of 2^20, 256 of 65536),
# the longest two-pass length, radix-stage lengths (two buffers of N each:
# 2^23 is the longest that fits, one segment per sub-batch) and length 1
CASES = [(4096, 40, 24), (1000, 33, 7), (1 << 16, 600, 300), (1 << 20, 40, 17),
         (1 << 22, 5, 3), (1 << 23, 2, 1), (3 ** 9, 30, 11), (1, 64, 3)]


@pytest.mark.parametrize("n,b1,b2", CASES)
@pytest.mark.parametrize("direction", [fs.FORWARD, fs.INVERSE])
def test_noalloc_matches_plan(n, b1, b2, direction):
    import torch
    announce("noalloc n=%d batches %d then %d dir=%d" % (n, b1, b2, direction))
    x = noise(n, b1, seed=31 + n % 97)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    sh = torch.cuda.current_stream().cuda_stream
    for b in (b1, b2):
        want = torch.zeros(b * n, dtype=torch.complex64, device="cuda")
        got = torch.full((b * n,), complex(7, 7), dtype=torch.complex64, device="cuda")
        with fs.Plan(n, b, direction) as p:
            p.exec_ptr(xd.data_ptr(), want.data_ptr(), sh)
        _noalloc(n, b, direction, xd.data_ptr(), got.data_ptr(), sh)
        torch.cuda.synchronize()
        g = got.cpu().numpy().reshape(b, n)
        w = want.cpu().numpy().reshape(b, n)
        e = oracle.rel_l2(g, w.astype(np.complex128))
        bound = oracle.tolerance(max(n, 2))
        print("  batch %d: max rel-L2 vs plan %.3e (bound %.3e)" % (b, e.max(), bound),
              flush=True)
        assert np.all(e <= bound), (b, float(e.max()))
        if n > 1 << 20:
            continue  # plan agreement only: the oracle takes seconds per segment here
        k = min(b, 3)
        ref = oracle.fft_recursive(x[:k], n, direction) if n > 1 else x[:k].astype(np.complex128)
        eo = oracle.rel_l2(g[:k], ref)
        assert np.all(eo <= bound), (b, float(eo.max()))


def test_noalloc_in_place_and_off_line():
    """In place, and with bases off a 128-byte line (the shifted two-pass
    forms place Y at the input's offset within a line)."""
    import torch
    n, b = 1 << 16, 20
    announce("noalloc in place / off line")
    x = noise(n, b + 1, seed=41)
    flat = x.reshape(-1)
    sh = torch.cuda.current_stream().cuda_stream
    for lead_in, lead_out in ((0, 0), (3, 5), (8, 0)):
        xd = torch.from_numpy(flat).cuda()
        yd = torch.zeros(b * n + 32, dtype=torch.complex64, device="cuda")
        _noalloc(n, b, fs.FORWARD, xd.data_ptr() + 8 * lead_in, yd.data_ptr() + 8 * lead_out, sh)
        torch.cuda.synchronize()
        got = yd.cpu().numpy()[lead_out:lead_out + b * n].reshape(b, n)
        src = flat[lead_in:lead_in + b * n].reshape(b, n)
        e = oracle.rel_l2(got[[0, b - 1]], oracle.fft_recursive(src[[0, b - 1]], n))
        assert np.all(e <= oracle.tolerance(n)), (lead_in, lead_out, e)
    xd = torch.from_numpy(flat[:b * n].copy()).cuda()
    _noalloc(n, b, fs.FORWARD, xd.data_ptr(), xd.data_ptr(), sh)
    torch.cuda.synchronize()
    got = xd.cpu().numpy().reshape(b, n)
    e = oracle.rel_l2(got[[0, b - 1]], oracle.fft_recursive(x[[0, b - 1]], n))
    assert np.all(e <= oracle.tolerance(n))


def test_noalloc_rejects_bad_arguments():
    import torch
    announce("noalloc argument checks")
    xd = torch.zeros(1 << 24, dtype=torch.complex64, device="cuda")
    for args, name in (((0, 1, -1), "FFT_ERR_INVALID_ARG"),
                       ((4096, 1, 3), "FFT_ERR_INVALID_ARG"),
                       ((7 * 64, 1, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),
                       ((1 << 25, 1, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),
                       ((1 << 24, 1, -1), "FFT_ERR_UNSUPPORTED_LENGTH")):
        with pytest.raises(fs.FFTError) as e:
            _noalloc(*args, xd.data_ptr(), xd.data_ptr(), 0)
        assert e.value.name == name, (args, e.value)
