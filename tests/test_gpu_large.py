"""Parity at the full 4096-point x 262144-segment size (2^30 samples,
8 GiB per buffer), in the launch configuration the benchmark times:
sampled segments against the FP64 oracle, Parseval on every segment, and
the inverse round trip."""
import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
from siggen import workloads

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def test_large_workload_full_size():
    import torch
    n, b = workloads.LARGE["seg_len"], workloads.LARGE["batch"]
    announce("large workload: generating %d x %d on the host" % (b, n))
    sig = workloads.large_signal()
    x = sig.segments(0, b)
    announce("large workload: forward + inverse on the GPU")
    xd = torch.from_numpy(x.reshape(-1)).to("cuda")
    fwd = fs.Plan(n, b, fs.FORWARD)
    inv = fs.Plan(n, b, fs.INVERSE)
    y = fwd.exec(xd)
    z = inv.exec(y)
    torch.cuda.synchronize()
    # sampled segments vs the oracle (first, last and a seeded sample)
    rng = np.random.default_rng(42)
    idx = np.unique(np.concatenate([[0, b - 1], rng.choice(b, 254, replace=False)]))
    ysamp = y.view(b, n)[torch.from_numpy(idx).to("cuda")].cpu().numpy()
    err = oracle.rel_l2(ysamp, oracle.fft_recursive(x[idx], n))
    print("  sampled %d segments: max rel-L2 %.3e mean %.3e" % (len(idx), err.max(), err.mean()))
    assert np.all(err <= oracle.tolerance(n))
    # Parseval on every segment (energies in FP64)
    xv = xd.view(b, n)
    ex = (xv.real.double() ** 2 + xv.imag.double() ** 2).sum(1)
    yv = y.view(b, n)
    ey = (yv.real.double() ** 2 + yv.imag.double() ** 2).sum(1)
    rel = ((ey - n * ex).abs() / (n * ex)).max().item()
    print("  Parseval over all %d segments: max rel deviation %.3e" % (b, rel))
    assert rel <= 2 * oracle.tolerance(n)
    # inverse round trip: z / N vs x, every segment
    zv = z.view(b, n)
    num = ((zv / n - xv).abs().double() ** 2).sum(1).sqrt()
    den = ex.sqrt()
    rt = (num / den).max().item()
    print("  round trip over all segments: max rel-L2 %.3e" % rt)
    assert rt <= 2 * oracle.tolerance(n)
    # the eight tones sit at their bins in every segment
    mags = yv[:, [t[0] for t in sig.tones]].abs()
    amps = torch.tensor([t[1] for t in sig.tones], device="cuda") * n
    assert ((mags - amps).abs().max() < 6 * np.sqrt(n)).item()
    fwd.close()
    inv.close()
