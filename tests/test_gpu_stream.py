"""Streaming through pinned host slots (fill -> H2D -> transform -> D2H ->
drain): every chunk against the oracle, callback failures, caller-owned
pinned buffers."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
import siggen

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def host_view(ptr, nbytes):
    buf = (ctypes.c_char * nbytes).from_address(ptr)
    return np.frombuffer(buf, dtype=np.complex64)


def run_stream(n, batch, n_chunks, sig, n_slots=3, fail_fill=None, fail_drain=None,
               native_fill=False):
    got = {}

    def fill(c, ptr, nbytes):
        if c == fail_fill:
            return 5
        sig.fill_ptr(c * batch * n, batch * n, ptr)
        return 0

    def drain(c, ptr, nbytes):
        if c == fail_drain:
            return 9
        got[c] = host_view(ptr, nbytes).copy().reshape(batch, n)
        return 0

    plan = fs.Plan(n, batch)
    if native_fill:
        src = sig.chunk_source(0, batch * n)
        rc, failed, st = plan.exec_stream(n_chunks, src, drain, n_slots)
    else:
        rc, failed, st = plan.exec_stream(n_chunks, fill, drain, n_slots)
    plan.close()
    return rc, failed, st, got


@pytest.mark.parametrize("n,batch,n_chunks,n_slots", [(4096, 64, 7, 3), (1000, 50, 4, 2),
                                                      (1 << 16, 3, 5, 3)])
def test_stream_every_chunk(n, batch, n_chunks, n_slots):
    announce("stream n=%d batch=%d chunks=%d slots=%d" % (n, batch, n_chunks, n_slots))
    sig = siggen.Signal(seed=99, seg_len=n, sigma=1.0, tones=[(7, 0.5, 0.0)])
    rc, failed, st, got = run_stream(n, batch, n_chunks, sig, n_slots)
    assert rc == 0 and failed is None
    assert st["chunks_done"] == n_chunks and sorted(got) == list(range(n_chunks))
    assert st["bytes_h2d"] == n_chunks * batch * n * 8
    for c in range(n_chunks):
        x = sig.segments(c * batch, batch)
        err = oracle.rel_l2(got[c], oracle.fft_recursive(x, n))
        assert np.all(err <= oracle.tolerance(n)), (c, err.max())


def test_stream_native_fill_and_chirp():
    n, batch, chunks = 1 << 20, 2, 3
    announce("stream 2^20 native fill")
    sig = siggen.Signal(seed=5, seg_len=n, sigma=0.0, chirp_amp=1.0)
    rc, failed, st, got = run_stream(n, batch, chunks, sig, 3, native_fill=True)
    assert rc == 0 and st["chunks_done"] == chunks
    t = np.arange(n, dtype=np.int64)
    want = np.sqrt(n) * np.exp(1j * np.pi / 4) * np.exp(-1j * np.pi * ((t * t) % (2 * n)) / n)
    for c in range(chunks):
        for s in range(batch):
            assert oracle.rel_l2(got[c][s][None], want[None])[0] <= oracle.tolerance(n)


@pytest.mark.parametrize("where", ["fill", "drain"])
def test_stream_callback_failure_reports_chunk(where):
    n, batch, chunks = 1024, 16, 8
    announce("stream failure in %s" % where)
    sig = siggen.Signal(seed=1, seg_len=n, sigma=1.0)
    kw = {"fail_fill": 5} if where == "fill" else {"fail_drain": 3}
    rc, failed, st, got = run_stream(n, batch, chunks, sig, 3, **kw)
    assert rc == -7  # FFT_ERR_CALLBACK
    bad = 5 if where == "fill" else 3
    assert failed == bad
    # every chunk below the failing one was handed out, correct
    assert sorted(got) == list(range(bad))
    for c in range(bad):
        x = sig.segments(c * batch, batch)
        assert np.all(oracle.rel_l2(got[c], oracle.fft_recursive(x, n)) <= oracle.tolerance(n))
    # the pipeline is reusable after a failure: resume from the failed chunk
    rc2, failed2, st2, got2 = run_stream(n, batch, 2, sig, 3)
    assert rc2 == 0 and failed2 is None


def test_stream_pinned_buffers():
    import torch
    n, batch, chunks = 4096, 32, 6
    announce("stream pinned")
    sig = siggen.Signal(seed=3, seg_len=n, sigma=1.0)
    ins = [torch.from_numpy(sig.segments(c * batch, batch).reshape(-1)).pin_memory()
           for c in range(chunks)]
    outs = [torch.empty(batch * n, dtype=torch.complex64).pin_memory() for _ in range(chunks)]
    plan = fs.Plan(n, batch)
    st = plan.exec_stream_pinned(chunks, [t.data_ptr() for t in ins],
                                 [t.data_ptr() for t in outs], 3)
    plan.close()
    assert st["chunks_done"] == chunks
    for c in range(chunks):
        x = ins[c].numpy().reshape(batch, n)
        y = outs[c].numpy().reshape(batch, n)
        assert np.all(oracle.rel_l2(y, oracle.fft_recursive(x, n)) <= oracle.tolerance(n))


def test_stream_configured_long_shape_every_segment():
    """The streamed 2^20-point workload at its configured chunk shape (512
    segments, 4 GiB per chunk), 3 chunks generated from the seed by the
    native producer: Parseval on every one of the 1536 segments and the
    oracle on the first and last segment of each chunk."""
    from siggen import workloads
    n, seg, chunks = workloads.LONG["seg_len"], workloads.LONG["chunk_segments"], 3
    announce("stream configured 2^20 x 512 per chunk, %d chunks" % chunks)
    sig = workloads.long_signal()
    fill, drain, src, chk = sig.checked_chunk_source(seg, chunks)
    with fs.Plan(n, seg) as plan:
        rc, failed, st = plan.exec_stream(chunks, (fill, src), (drain, src), 3)
    assert rc == 0 and failed is None and st["chunks_done"] == chunks
    tol = oracle.tolerance(n)
    dev = np.abs(chk.energy_out / (n * chk.energy_in) - 1.0)
    print("  parseval max rel dev %.3e over %d segments" % (dev.max(), dev.size), flush=True)
    assert dev.size == chunks * seg and np.all(dev <= 2 * tol + tol * tol)
    # the kept first and last segments, against the oracle
    idx = [c * seg + s for c in range(chunks) for s in (0, seg - 1)]
    x = np.concatenate([sig.segments(i, 1) for i in idx])
    err = oracle.rel_l2(chk.saved_out.reshape(-1, n), oracle.fft_recursive(x, n))
    print("  oracle max rel-L2 %.3e on %d segments" % (err.max(), len(idx)), flush=True)
    assert np.all(err <= tol)


def test_stream_library_pinned_buffers():
    n, batch, chunks, pool = 1 << 16, 8, 5, 2
    announce("stream library pinned buffers")
    sig = siggen.Signal(seed=8, seg_len=n, sigma=1.0, chirp_amp=0.5)
    nbytes = batch * n * 8
    ins = [fs.HostBuffer(nbytes) for _ in range(pool)]
    outs = [fs.HostBuffer(nbytes) for _ in range(pool)]
    try:
        for c in range(pool):
            sig.fill_ptr(c * batch * n, batch * n, ins[c].ptr)
        with fs.Plan(n, batch) as plan:
            assert plan.stream_timeline() == []
            st = plan.exec_stream_pinned(chunks, [b.ptr for b in ins], [b.ptr for b in outs], 3)
            tl = plan.stream_timeline()
        assert st["chunks_done"] == chunks
        # one entry per chunk, each chunk's steps in order on the GPU clock,
        # copies in issued in chunk order
        assert [t["chunk"] for t in tl] == list(range(chunks))
        assert tl[0]["h2d_start_ms"] >= 0.0
        for t in tl:
            seq = [t["h2d_start_ms"], t["h2d_end_ms"], t["compute_start_ms"],
                   t["compute_end_ms"], t["d2h_start_ms"], t["d2h_end_ms"]]
            assert all(a <= b for a, b in zip(seq, seq[1:])), t
        for a, b in zip(tl, tl[1:]):
            assert a["h2d_end_ms"] <= b["h2d_start_ms"]
        for c in range(pool):
            x = ins[c].view().reshape(batch, n).copy()
            y = outs[c].view().reshape(batch, n).copy()
            assert np.all(oracle.rel_l2(y, oracle.fft_recursive(x, n)) <= oracle.tolerance(n))
    finally:
        for b in ins + outs:
            b.close()
