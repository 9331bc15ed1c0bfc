"""Helpers shared by the GPU tests: run the library on host arrays and
compare with the oracle.  Every case prints its name before touching the
GPU, so a failing run names the case."""
import sys

import numpy as np

import oracle
import paper_1407_6915_amd as fs
import siggen


def announce(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def noise(n, batch, seed=1234, stream=0):
    return siggen.Signal(seed=seed, seg_len=n, sigma=1.0, stream=stream).segments(0, batch)


def run(n, x, direction=fs.FORWARD, variant=None, inplace=False):
    """Transform host complex64 [batch, n] through the C ABI; returns host array."""
    import torch
    x = np.ascontiguousarray(x, dtype=np.complex64).reshape(-1, n)
    b = x.shape[0]
    xd = torch.from_numpy(x.reshape(-1)).to("cuda")
    with fs.Plan(n, b, direction, variant) as p:
        if inplace:
            p.exec(xd, xd)
            y = xd
        else:
            y = p.exec(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy().reshape(b, n)


def check(n, got, x, direction=fs.FORWARD, tol=None, what=""):
    ref = oracle.fft_recursive(x, n, direction)
    err = oracle.rel_l2(got, ref)
    bound = oracle.tolerance(n) if tol is None else tol
    print("  %s n=%d batch=%d max rel-L2 %.3e mean %.3e (bound %.3e)"
          % (what, n, len(err), err.max(), err.mean(), bound), flush=True)
    assert np.all(err <= bound), (what, n, float(err.max()), int(err.argmax()))
    return err
