"""The persistent work-list kernel on uneven batches: every segment against
the oracle, in place, graph replay, agreement with plain per-length plans,
and the full 200000-segment uneven workload on sampled segments."""
import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
import siggen
from siggen import workloads

from gpu_helpers import announce

pytestmark = pytest.mark.gpu

LENGTHS = [256, 1000, 1024, 1536, 4096, 6000, 16384, 65536]


class routes:
    """Work-list routes forced through a tuning cache: {length: route}, 0 =
    the work-list kernel's tiles, 1 + k = the k-th indexed one-pass kernel
    (grid: its own).  Cleared on exit."""

    def __init__(self, table, tmp_path, grid=0):
        self.table, self.path, self.grid = table, str(tmp_path / "routes.json"), grid

    def __enter__(self):
        import json
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        ents = [{"n": n, "variant": -2, "grid_mult": 0, "wl_route": r, "wl_grid": self.grid}
                for n, r in self.table.items()]
        json.dump({"arch": arch, "entries": ents}, open(self.path, "w"))
        assert fs.tune_load(self.path) == len(ents)
        return self

    def __exit__(self, *exc):
        fs.tune_clear()


def packed(lengths, gap=0, seed=0):
    """Back-to-back layout in list order (optionally with gaps); returns
    in offsets, out offsets (a different permutation of slots) and total."""
    offs = np.zeros(len(lengths), np.int64)
    pos = 0
    for i, n in enumerate(lengths):
        offs[i] = pos
        pos += n + gap
    return offs, pos


def to_entries(in_off, out_off, lengths):
    arr = np.zeros(len(lengths), dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                                        ("segment_len", "<u4"), ("job", "<u4")])
    arr["in_off"], arr["out_off"], arr["segment_len"] = in_off, out_off, lengths
    arr["job"] = np.arange(len(lengths))
    return arr


def check_all(x_host, y_host, in_off, out_off, lengths, direction=fs.FORWARD, sample=None):
    idx = range(len(lengths)) if sample is None else sample
    worst = 0.0
    for i in idx:
        n = int(lengths[i])
        x = x_host[in_off[i]:in_off[i] + n]
        ref = oracle.fft_recursive(x, n, direction)
        e = oracle.rel_l2(y_host[out_off[i]:out_off[i] + n][None], ref)[0]
        assert e <= oracle.tolerance(n), (i, n, e)
        worst = max(worst, e / oracle.tolerance(n))
    print("  worst error / bound = %.3f" % worst, flush=True)


@pytest.mark.parametrize("direction", [fs.FORWARD, fs.INVERSE])
def test_mixed_lengths_every_segment(direction):
    import torch
    rng = np.random.default_rng(7)
    lengths = np.array(rng.choice(LENGTHS, 60).tolist() + LENGTHS, np.int64)
    rng.shuffle(lengths)
    announce("work list %d segments dir=%d" % (len(lengths), direction))
    in_off, total = packed(lengths, gap=3)
    # outputs in reverse order, in a buffer of their own
    out_off, out_total = packed(lengths[::-1])
    out_off = out_off[::-1].copy()
    x = siggen.Signal(seed=11, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(out_total, dtype=torch.complex64, device="cuda")
    with fs.WorkList(to_entries(in_off, out_off, lengths), direction) as wl:
        d = wl.describe()
        assert d["items"] == len(lengths)
        wl.exec(xd, yd)
        wl.status()
        y = yd.cpu().numpy()
        check_all(x, y, in_off, out_off, lengths, direction)
        # graph replay equals the eager launch, several replays with eager
        # work in between
        for _ in range(3):
            yd.zero_()
            wl.exec(xd, yd, graph=True)
            wl.status()
            assert np.array_equal(yd.cpu().numpy(), y)
            xd.add_(0)
    # agreement with plain per-length plans on the same segments
    for n in LENGTHS:
        sel = np.nonzero(lengths == n)[0]
        seg = np.stack([x[in_off[i]:in_off[i] + n] for i in sel])
        xs = torch.from_numpy(seg.reshape(-1)).cuda()
        with fs.Plan(n, len(sel), direction) as p:
            ys = p.exec(xs).cpu().numpy().reshape(len(sel), n)
        mine = np.stack([y[out_off[i]:out_off[i] + n] for i in sel])
        e = oracle.rel_l2(mine, ys.astype(np.complex128))
        assert np.all(e <= 2 * oracle.tolerance(n)), (n, e.max())


def test_wide_tiles_alone():
    """A list of only 16384-point segments: no work-list task at all, just
    the launch of wide tiles (one 512-thread workgroup per segment), out of
    place, replayed from a graph, and in place."""
    import torch
    lengths = np.full(37, 16384, np.int64)
    announce("work list of wide tiles only")
    in_off, total = packed(lengths, gap=5)
    out_off, out_total = packed(lengths[::-1])
    out_off = out_off[::-1].copy()
    x = siggen.Signal(seed=14, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(out_total, dtype=torch.complex64, device="cuda")
    with fs.WorkList(to_entries(in_off, out_off, lengths)) as wl:
        d = wl.describe()
        assert d["tasks"] == 0 and d["wide_segments"] == len(lengths)
        assert d["scratch_bytes"] == 0
        wl.exec(xd, yd)
        wl.status()
        y = yd.cpu().numpy()
        check_all(x, y, in_off, out_off, lengths)
        for _ in range(2):
            yd.zero_()
            wl.exec(xd, yd, graph=True)
            wl.status()
            assert np.array_equal(yd.cpu().numpy(), y)
    with fs.WorkList(to_entries(in_off, in_off, lengths)) as wl:
        wl.exec(xd, xd)
        wl.status()
    check_all(x, xd.cpu().numpy(), in_off, in_off, lengths)


@pytest.mark.parametrize("lead", [0, 8, 3, 13])
def test_two_pass_segments_at_any_line_offset(lead):
    """Two-pass segments (65536 and 2^20 points) whose inputs and outputs
    start at every kind of offset within a 128-byte line: the column and row
    blocks then start mid-segment and the last one wraps round."""
    import torch
    lengths = np.array([65536, 1 << 20, 65536, 65536], np.int64)
    announce("work list two-pass segments, lead %d samples" % lead)
    in_off, total = packed(lengths, gap=5)
    in_off = in_off + lead
    out_off, out_total = packed(lengths[::-1], gap=7)
    out_off = out_off[::-1].copy() + (lead * 3) % 16
    x = siggen.Signal(seed=15, seg_len=1, sigma=1.0).samples(0, total + lead)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(out_total + 16, dtype=torch.complex64, device="cuda")
    for direction in (fs.FORWARD, fs.INVERSE):
        with fs.WorkList(to_entries(in_off, out_off, lengths), direction) as wl:
            wl.exec(xd, yd)
            wl.status()
        check_all(x, yd.cpu().numpy(), in_off, out_off, lengths, direction)


def test_long_segments_go_through_the_plan_in_runs():
    """2^20-point entries run through a four-step plan, one call per run of
    consecutive entries whose inputs and outputs advance by one segment:
    runs of 3, 2 and 1 (the second starting inside a cache line), mixed with
    work-list lengths, in place and out of place; then graph replays across
    a reset whose longer run makes the plan grow (the old graph, which holds
    the old runs, must not be replayed)."""
    import torch
    m = 1 << 20
    lengths = np.array([m, m, m, 4096, m, m, 65536, m], np.int64)
    in_off = np.array([0, m, 2 * m, 3 * m, 3 * m + 4099, 4 * m + 4099, 5 * m + 4099,
                       5 * m + 4099 + 65536], np.int64)
    total = int(in_off[-1] + m)
    announce("work list 2^20 runs, %d samples" % total)
    x = siggen.Signal(seed=16, seg_len=1, sigma=1.0).samples(0, total)
    with fs.WorkList(to_entries(in_off, in_off, lengths)) as wl:
        assert wl.describe()["plan_runs"] == 3
        xd = torch.from_numpy(x).cuda()
        wl.exec(xd, xd)                                     # in place
        wl.status()
        check_all(x, xd.cpu().numpy(), in_off, in_off, lengths)
        # out of place, outputs in reverse slot order: no entry stays in a run
        out_off, out_total = packed(lengths[::-1], gap=3)
        out_off = out_off[::-1].copy()
        xd = torch.from_numpy(x).cuda()
        yd = torch.zeros(out_total, dtype=torch.complex64, device="cuda")
        wl.reset(to_entries(in_off, out_off, lengths))
        assert wl.describe()["plan_runs"] == 6
        wl.exec(xd, yd, graph=True)
        wl.exec(xd, yd, graph=True)
        wl.status()
        check_all(x, yd.cpu().numpy(), in_off, out_off, lengths, sample=[0, 4, 5, 6])
        # a run of 5 (longer than any before): the plan grows, the graph is
        # captured again
        lengths2 = np.array([m] * 5 + [1024], np.int64)
        off2 = np.concatenate([np.arange(5) * m, [5 * m]]).astype(np.int64)
        wl.reset(to_entries(off2, off2, lengths2))
        assert wl.describe()["plan_runs"] == 1
        yd.zero_()
        wl.exec(xd, yd, graph=True)
        wl.status()
        check_all(x, yd.cpu().numpy(), off2, off2, lengths2, sample=[0, 4, 5])


def test_failed_reset_refuses_to_run_until_the_next_reset():
    """A reset whose entries pass the checks but whose two-pass scratch
    cannot be allocated (600000 segments of 65536 points need 315 GB)
    returns FFT_ERR_OUT_OF_MEMORY; the work list then refuses to run,
    without a launch, until a reset succeeds."""
    import torch
    n = 1024
    announce("work list failed reset")
    x = siggen.Signal(seed=17, seg_len=n, sigma=1.0).samples(0, 4 * n)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(4 * n, dtype=torch.complex64, device="cuda")
    offs = np.arange(4, dtype=np.int64) * n
    small = to_entries(offs, offs, np.full(4, n, np.int64))
    big_n = 600000
    big_off = np.arange(big_n, dtype=np.int64) * 65536
    big = to_entries(big_off, big_off, np.full(big_n, 65536, np.int64))
    with fs.WorkList(small) as wl:
        with pytest.raises(fs.FFTError) as e:
            wl.reset(big)
        assert e.value.name == "FFT_ERR_OUT_OF_MEMORY"
        with pytest.raises(fs.FFTError) as e:
            wl.exec(xd, yd)
        assert e.value.name == "FFT_ERR_INVALID_ARG"
        wl.reset(small)
        wl.exec(xd, yd)
        wl.status()
    check_all(x, yd.cpu().numpy(), offs, offs, np.full(4, n, np.int64))


def test_in_place_and_overlap_rules():
    import torch
    lengths = np.array([4096, 65536, 256, 16384, 1000, 6000, 1536, 1024] * 3, np.int64)
    announce("work list in place")
    off, total = packed(lengths)
    x = siggen.Signal(seed=12, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    with fs.WorkList(to_entries(off, off, lengths)) as wl:
        wl.exec(xd, xd)
        wl.status()
    check_all(x, xd.cpu().numpy(), off, off, lengths)
    # two entries that swap places cannot run in place (each output lands
    # on the other's input), but can run out of place
    ent = to_entries(np.array([0, 4096]), np.array([4096, 0]), np.array([4096, 4096]))
    x2 = siggen.Signal(seed=13, seg_len=1, sigma=1.0).samples(0, 8192)
    xd2 = torch.from_numpy(x2).cuda()
    with fs.WorkList(ent) as wl:
        with pytest.raises(fs.FFTError) as e:
            wl.exec(xd2, xd2)
        assert e.value.name == "FFT_ERR_OVERLAP"
        yd2 = torch.zeros_like(xd2)
        wl.exec(xd2, yd2)
        wl.status()
    check_all(x2, yd2.cpu().numpy(), [0, 4096], [4096, 0], [4096, 4096])


def test_bounds_are_checked():
    """A work list reaching past the end of its buffer's allocation is
    refused.  The case runs only after the HIP runtime itself reports the
    raw allocation's exact extent, which is what the library's check reads,
    so no kernel can start on it."""
    import ctypes
    import torch
    announce("work list bounds")
    hip = ctypes.CDLL("libamdhip64.so")
    torch.cuda.synchronize()
    p = ctypes.c_void_p()
    nbytes = 1 << 20
    assert hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes)) == 0
    try:
        base, size = ctypes.c_void_p(), ctypes.c_size_t()
        rc = hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), p)
        if rc == 0 and base.value == p.value and size.value == nbytes:
            n_fit = nbytes // 8
            with fs.WorkList([(0, 0, 4096), (n_fit, n_fit, 4096)]) as wl:
                with pytest.raises(fs.FFTError) as e:
                    wl.exec_ptr(p.value, p.value, 0)
                assert e.value.name == "FFT_ERR_BOUNDS"
    finally:
        hip.hipFree(p)


def test_uneven_workload_full_size():
    import torch
    lengths = workloads.uneven_lengths()
    n_seg = len(lengths)
    in_off = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    total = int(lengths.sum())
    announce("uneven workload: %d segments, %d samples" % (n_seg, total))
    sig = workloads.uneven_signal()
    xd = torch.empty(total, dtype=torch.complex64, device="cuda")
    chunk = 1 << 27
    for a in range(0, total, chunk):
        m = min(chunk, total - a)
        xd[a:a + m].copy_(torch.from_numpy(sig.samples(a, m)))
    yd = torch.empty_like(xd)
    with fs.WorkList(to_entries(in_off, in_off, lengths)) as wl:
        wl.exec(xd, yd)
        wl.status()
    rng = np.random.default_rng(4)
    worst = 0.0
    for n in workloads.UNEVEN_LENGTHS:
        sel = rng.choice(np.nonzero(lengths == n)[0], 16, replace=False)
        for i in sel:
            a = int(in_off[i])
            x = sig.samples(a, n)
            y = yd[a:a + n].cpu().numpy()
            e = oracle.rel_l2(y[None], oracle.fft_recursive(x, n))[0]
            assert e <= oracle.tolerance(n), (n, i, e)
            worst = max(worst, e / oracle.tolerance(n))
    print("  sampled 16 per length, worst error / bound %.3f" % worst, flush=True)


@pytest.mark.parametrize("route", [1, 2])
def test_indexed_routes_walk_several_segments(route, tmp_path):
    """The indexed one-pass launches on a grid of one resident wave of
    workgroups (wl_grid 1), over enough segments of each length that every
    workgroup transforms several tiles in turn; the 65536-point segments
    through the indexed passes at the same grid.  Sampled segments of every
    length (the first, the last and 40 drawn) against the oracle."""
    import torch
    counts = {256: 40000, 1000: 12000, 1536: 8000, 4096: 3000, 6000: 2000, 65536: 20}
    rng = np.random.default_rng(40 + route)
    lengths = np.concatenate([np.full(c, n, np.int64) for n, c in counts.items()])
    rng.shuffle(lengths)
    in_off, total = packed(lengths, gap=1)
    announce("indexed routes=%d on one resident wave, %d segments" % (route, len(lengths)))
    x = siggen.Signal(seed=41, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(total, dtype=torch.complex64, device="cuda")
    table = {n: (route if n != 65536 else 1) for n in counts}
    with routes(table, tmp_path, grid=1), fs.WorkList(to_entries(in_off, in_off, lengths)) as wl:
        d = wl.describe()
        assert d["indexed_two_pass_segments"] == counts[65536]
        wl.exec(xd, yd)
        wl.status()
    y = yd.cpu().numpy()
    sample = []
    for n in counts:
        idx = np.nonzero(lengths == n)[0]
        sample += [int(idx[0]), int(idx[-1])] + [int(i) for i in rng.choice(idx, 40)]
    check_all(x, y, in_off, in_off, lengths, sample=sample)


@pytest.mark.parametrize("route", [0, 1, 2])
def test_one_pass_routes(route, tmp_path):
    """Every one-pass length through the work-list kernel's tiles (0), its
    default indexed kernel (1) or its second indexed kernel (2, where the
    length has one): every segment against the oracle, eager and graph."""
    import torch
    one_pass = [256, 1000, 1024, 1536, 4096, 6000]
    rng = np.random.default_rng(30 + route)
    lengths = np.array(rng.choice(LENGTHS, 50).tolist() + LENGTHS, np.int64)
    rng.shuffle(lengths)
    in_off, total = packed(lengths, gap=5)
    out_off, out_total = packed(lengths[::-1], gap=1)
    out_off = out_off[::-1].copy()
    announce("work list routes=%d, %d segments" % (route, len(lengths)))
    x = siggen.Signal(seed=31, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(out_total, dtype=torch.complex64, device="cuda")
    # 65536: its tasks (route 0) or its indexed passes (routes 1, 2 -> 1)
    table = {n: route for n in one_pass}
    table[65536] = min(route, 1)
    with routes(table, tmp_path):
        with fs.WorkList(to_entries(in_off, out_off, lengths)) as wl:
            d = wl.describe()
            assert d["indexed_two_pass_segments"] == (0 if route == 0 else
                                                      int((lengths == 65536).sum()))
            if route == 0:
                assert d["indexed_launches"] == 0
            else:
                assert set(d["indexed"]) == {str(n) for n in one_pass}
                for n in one_pass:
                    want = route - 1 if route - 1 < fs.indexed_count(n) else 0
                    assert d["indexed"][str(n)]["candidate"] == want
            wl.exec(xd, yd)
            wl.status()
            y = yd.cpu().numpy()
            check_all(x, y, in_off, out_off, lengths)
            for _ in range(2):
                yd.zero_()
                wl.exec(xd, yd, graph=True)
                wl.status()
                assert np.array_equal(yd.cpu().numpy(), y)


def test_graph_recaptured_when_a_reset_changes_launch_arguments(tmp_path):
    """The graph's launches hold the task counts and splits, the wide range
    and the grids as fixed arguments.  Resets that keep the planned runs and
    the grid but change those must not replay the old graph: (1) a 4096-point
    segment added after a lone 2^20-point run (the old graph has no
    work-list launch at all); (2) two lists with the same task count, hence
    the same grid, but a different split between the two launches."""
    import torch
    m = 1 << 20
    announce("work list graph key: added task after a planned run")
    x = siggen.Signal(seed=18, seg_len=1, sigma=1.0).samples(0, m + 4096)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(m + 4096, dtype=torch.complex64, device="cuda")
    with fs.WorkList(to_entries([0], [0], [m])) as wl:
        wl.exec(xd, yd, graph=True)
        wl.status()
        check_all(x, yd.cpu().numpy(), [0], [0], [m])
        wl.reset(to_entries([0, m], [0, m], [m, 4096]))
        yd.zero_()
        wl.exec(xd, yd, graph=True)
        wl.status()
        check_all(x, yd.cpu().numpy(), [0, m], [0, m], [m, 4096])

    announce("work list graph key: same task count, other split")
    s = 65536

    def layout(n_two, n_short):
        lengths = np.array([s] * n_two + [256] * n_short, np.int64)
        off, total = packed(lengths)
        return lengths, off, total

    l1, o1, t1 = layout(2, 32 * 10)     # 64 two-pass + 10 one-pass tasks
    l2, o2, t2 = layout(1, 32 * 42)     # 32 two-pass + 42 one-pass tasks
    total = max(t1, t2)
    x = siggen.Signal(seed=19, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(total, dtype=torch.complex64, device="cuda")
    # the 256- and 65536-point segments as work-list tasks (not launches
    # of their own)
    with routes({256: 0, 65536: 0}, tmp_path), fs.WorkList(to_entries(o1, o1, l1)) as wl:
        d1 = wl.describe()
        wl.exec(xd, yd, graph=True)
        wl.status()
        check_all(x, yd.cpu().numpy(), o1, o1, l1, sample=[0, 1, 2, len(l1) - 1])
        wl.reset(to_entries(o2, o2, l2))
        d2 = wl.describe()
        assert d1["tasks"] == d2["tasks"] and d1["grid"] == d2["grid"]
        assert d1["first_launch_tasks"] != d2["first_launch_tasks"]
        yd.zero_()
        wl.exec(xd, yd, graph=True)
        wl.status()
        y_graph = yd.cpu().numpy()
        yd.zero_()
        wl.exec(xd, yd)
        wl.status()
        assert np.array_equal(y_graph, yd.cpu().numpy())
        check_all(x, y_graph, o2, o2, l2, sample=[0, 1, 500, len(l2) - 1])


def test_one_call_worklist():
    """fft_exec_worklist(items, n, direction, in_base, out_base, stream):
    each call builds nothing the caller sees; two calls in a row on one
    stream (the second list smaller), then a call on another stream, and
    the inverse direction, all against the oracle."""
    import torch
    rng = np.random.default_rng(21)
    lengths = np.array(rng.choice(LENGTHS, 40).tolist() + LENGTHS + [1 << 20], np.int64)
    rng.shuffle(lengths)
    in_off, total = packed(lengths, gap=1)
    out_off, out_total = packed(lengths[::-1], gap=2)
    out_off = out_off[::-1].copy()
    announce("one-call work list, %d segments" % len(lengths))
    x = siggen.Signal(seed=20, seg_len=1, sigma=1.0).samples(0, total)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros(out_total, dtype=torch.complex64, device="cuda")
    try:
        fs.exec_worklist(to_entries(in_off, out_off, lengths), xd, yd)
        torch.cuda.synchronize()
        check_all(x, yd.cpu().numpy(), in_off, out_off, lengths)
        k = len(lengths) // 3
        yd.zero_()
        fs.exec_worklist(to_entries(in_off[:k], out_off[:k], lengths[:k]), xd, yd)
        torch.cuda.synchronize()
        check_all(x, yd.cpu().numpy(), in_off[:k], out_off[:k], lengths[:k])
        side = torch.cuda.Stream()
        yd.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            fs.exec_worklist(to_entries(in_off, out_off, lengths), xd, yd, fs.INVERSE)
        side.synchronize()
        check_all(x, yd.cpu().numpy(), in_off, out_off, lengths, fs.INVERSE)
        with pytest.raises(fs.FFTError) as e:
            fs.exec_worklist(to_entries([0], [0], [7]), xd, yd)
        assert e.value.name == "FFT_ERR_UNSUPPORTED_LENGTH"
    finally:
        fs.worklist_cache_clear()
