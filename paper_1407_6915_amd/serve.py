"""Continuous-batching FFT server over the work-list kernel.

Jobs (``n_seg`` segments of ``seg_len`` samples) arrive over time.  The
loop admits them in arrival order while a device arena of bounded size
(the HBM budget) has room, copies each admitted job in on a copy stream,
and whenever the transform stream is free packs the segments of EVERY job
whose input has landed -- whatever their lengths and jobs -- into one
work-list launch.  Finished jobs go back to the host on a third stream and
release their arena space, so jobs that arrive while others are on the GPU
are admitted as memory frees up and their copies overlap other jobs'
transforms.  Each segment is computed by the same per-length routine
whatever it is packed with, so a job's result does not depend on the mix.

The scheduler is written against a small executor interface: ``GpuExecutor``
drives the library; ``SimExecutor`` replays the same decisions on a virtual
clock with modelled copy and transform times (used to test the scheduler
on a host without a GPU).
"""
from __future__ import annotations

import bisect
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

FORWARD = -1

SAMPLE_BYTES = 8
ALIGN = 64  # samples (512 bytes) per arena slot boundary


class Arena:
    """First-fit allocator over ``capacity`` samples (offsets in samples)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free: List[List[int]] = [[0, self.capacity]]  # sorted [start, size]
        self.used = 0

    def alloc(self, n: int) -> Optional[int]:
        n = -(-int(n) // ALIGN) * ALIGN
        for i, (start, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    self.free.pop(i)
                else:
                    self.free[i] = [start + n, size - n]
                self.used += n
                return start
        return None

    def release(self, start: int, n: int) -> None:
        n = -(-int(n) // ALIGN) * ALIGN
        self.used -= n
        i = bisect.bisect_left(self.free, [start, 0])
        self.free.insert(i, [start, n])
        # merge with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i][1] += self.free.pop(i + 1)[1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1][1] += self.free.pop(i)[1]

    def fits_ever(self, n: int) -> bool:
        return -(-int(n) // ALIGN) * ALIGN <= self.capacity


@dataclass
class JobState:
    index: int
    arrival_s: float
    seg_len: int
    n_seg: int
    host_in: int = 0      # host address of the payload (pinned)
    host_out: int = 0     # host address for the spectra (pinned)
    off: int = -1         # arena offset (samples); transformed in place
    admitted_s: float = math.nan
    done_s: float = math.nan
    launch: int = -1      # which packed launch computed it
    status: str = "pending"
    tokens: Dict[str, object] = field(default_factory=dict)

    @property
    def samples(self) -> int:
        return self.seg_len * self.n_seg


class SimExecutor:
    """Virtual-clock stand-in for the GPU: three in-order streams with
    modelled durations (host link and HBM bandwidths, launch overhead)."""

    def __init__(self, link_gbs=50.0, hbm_gbs=5000.0, launch_us=10.0):
        self.t = 0.0
        self.link = link_gbs * 1e9
        self.hbm = hbm_gbs * 1e9
        self.launch = launch_us * 1e-6
        self.busy = {"in": 0.0, "comp": 0.0, "out": 0.0}
        self.ends: List[float] = []           # completion times not yet reached
        self.launches: List[List[int]] = []  # job indices per compute launch
        self.issued: List[float] = []        # clock time each launch was issued
        self.max_launch_samples = 0

    def now(self) -> float:
        return self.t

    def _enqueue(self, stream, dur, after=0.0):
        start = max(self.t, self.busy[stream], after)
        self.busy[stream] = start + dur
        bisect.insort(self.ends, self.busy[stream])
        return self.busy[stream]

    def h2d(self, job: JobState):
        return self._enqueue("in", job.samples * SAMPLE_BYTES / self.link)

    def compute(self, jobs: List[JobState], after=None):
        samples = sum(j.samples for j in jobs)
        self.max_launch_samples = max(self.max_launch_samples, samples)
        self.launches.append([j.index for j in jobs])
        self.issued.append(self.t)
        passes = sum(j.samples * (2 if j.seg_len > 16384 else 1) for j in jobs)
        return self._enqueue("comp", self.launch + 16.0 * passes / self.hbm,
                             0.0 if after is None else after)

    def d2h(self, job: JobState, after):
        return self._enqueue("out", job.samples * SAMPLE_BYTES / self.link, after)

    def done(self, token) -> bool:
        return token <= self.t + 1e-12

    def stream_idle(self) -> bool:
        return self.busy["comp"] <= self.t + 1e-12

    def advance(self, until: float) -> None:
        """Move the clock to the next completion or `until`, whichever first."""
        while self.ends and self.ends[0] <= self.t + 1e-12:
            self.ends.pop(0)
        nxt = min(self.ends[0] if self.ends else math.inf, until)
        if nxt < math.inf:
            self.t = max(self.t, nxt)

    def finish_time(self, token) -> float:
        return token


class GpuExecutor:
    """Runs the schedule on the GPU through the library: one device arena,
    three torch streams (copy in, transform, copy out), one reusable work
    list re-filled for every packed launch."""

    def __init__(self, arena_samples: int = 0, direction: int = FORWARD, device: str = "cuda",
                 max_launch_samples: int = 0, hbm_budget_bytes: int = 0):
        """arena_samples: size of the job arena; or hbm_budget_bytes: the
        whole device footprint allowed, of which the arena gets what the
        work list's reserved arrays, scratch and plan leave."""
        import torch
        from . import WorkList
        self.torch = torch
        self.dev = torch.device(device)
        self.s_in = torch.cuda.Stream(self.dev)
        self.s_comp = torch.cuda.Stream(self.dev)
        self.s_out = torch.cuda.Stream(self.dev)
        self.wl = WorkList((), direction)
        if max_launch_samples:
            self.reserve(max_launch_samples)
        self.resident_bytes = int(self.wl.describe().get("device_bytes", 0))
        if hbm_budget_bytes:
            arena_samples = (hbm_budget_bytes - self.resident_bytes) // SAMPLE_BYTES
            if arena_samples <= 0:
                raise ValueError("the work list's %d resident bytes exceed the budget"
                                 % self.resident_bytes)
        self.arena_samples = int(arena_samples)
        self.arena = torch.empty(self.arena_samples, dtype=torch.complex64, device=self.dev)
        self.base = self.arena.data_ptr()
        self.t0 = time.perf_counter()
        self.launches: List[List[int]] = []
        self.max_launch_samples = 0
        self._comp_ev = None

    def reserve(self, max_launch_samples: int) -> None:
        """Grow the work list's device arrays to what a launch of up to
        max_launch_samples can need (task and item lists of the shortest
        length, the two-pass scratch of 65536-point segments, the four-step
        plan of the 2^20-point ones), so that no later reset has to
        synchronise the device and reallocate while jobs are in flight.
        Only the capacities are kept."""
        import numpy as np
        from . import worklist_supported
        lens = [n for n in (256, 1000, 1024, 1536, 4096, 6000, 16384, 65536, 1 << 20)
                if worklist_supported(n)]
        for n in sorted({min(lens), 65536, max(lens)} & set(lens)):
            cnt = max(1, max_launch_samples // n)
            ent = np.zeros(cnt, dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                                       ("segment_len", "<u4"), ("job", "<u4")])
            ent["in_off"] = ent["out_off"] = np.arange(cnt, dtype=np.uint64) * np.uint64(n)
            ent["segment_len"] = n
            self.wl.reset(ent, stream=self.s_comp.cuda_stream)
        self.wl.reset((), stream=self.s_comp.cuda_stream)
        self.torch.cuda.synchronize(self.dev)

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def _copy(self, stream, dst, src, nbytes, after=None):
        torch = self.torch
        import ctypes
        hip = _hip()
        with torch.cuda.stream(stream):
            if after is not None:
                stream.wait_event(after)
            kind = 1 if dst == "h2d" else 2  # hipMemcpyHostToDevice / DeviceToHost
            rc = hip.hipMemcpyAsync(ctypes.c_void_p(src[0]), ctypes.c_void_p(src[1]),
                                    ctypes.c_size_t(nbytes), kind,
                                    ctypes.c_void_p(stream.cuda_stream))
            if rc != 0:
                raise RuntimeError("hipMemcpyAsync failed (%d)" % rc)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def h2d(self, job: JobState):
        dst = self.base + job.off * SAMPLE_BYTES
        return self._copy(self.s_in, "h2d", (dst, job.host_in), job.samples * SAMPLE_BYTES)

    def compute(self, jobs: List[JobState], after=None):
        import numpy as np
        torch = self.torch
        n = sum(j.n_seg for j in jobs)
        ent = np.zeros(n, dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                                 ("segment_len", "<u4"), ("job", "<u4")])
        k = 0
        for j in jobs:
            offs = j.off + np.arange(j.n_seg, dtype=np.uint64) * np.uint64(j.seg_len)
            ent["in_off"][k:k + j.n_seg] = offs
            ent["out_off"][k:k + j.n_seg] = offs
            ent["segment_len"][k:k + j.n_seg] = j.seg_len
            ent["job"][k:k + j.n_seg] = j.index
            k += j.n_seg
        self.launches.append([j.index for j in jobs])
        self.max_launch_samples = max(self.max_launch_samples, sum(j.samples for j in jobs))
        sh = self.s_comp.cuda_stream
        if after is not None:
            self.s_comp.wait_event(after)  # e.g. the job's own input copy
        self.wl.reset(ent, stream=sh)
        self.wl.exec_ptr(self.base, self.base, sh)
        ev = torch.cuda.Event()
        ev.record(self.s_comp)
        self._comp_ev = ev
        return ev

    def d2h(self, job: JobState, after):
        src = self.base + job.off * SAMPLE_BYTES
        return self._copy(self.s_out, "d2h", (job.host_out, src), job.samples * SAMPLE_BYTES,
                          after=after)

    def done(self, token) -> bool:
        return token.query()

    def stream_idle(self) -> bool:
        return self._comp_ev is None or self._comp_ev.query()

    def advance(self, until: float) -> None:
        # nothing to do on the host right now: yield briefly
        dt = until - self.now()
        time.sleep(min(max(dt, 0.0), 50e-6))

    def finish(self) -> None:
        self.torch.cuda.synchronize(self.dev)
        self.wl.status(self.s_comp.cuda_stream)


_HIP = None


def _hip():
    global _HIP
    if _HIP is None:
        import ctypes
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpyAsync.restype = ctypes.c_int
        _HIP.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
    return _HIP


class RejectedJob(Exception):
    pass


def serve(jobs: List[JobState], executor, arena_samples: int,
          max_launch_samples: int = 1 << 31, reject_oversized: bool = True,
          max_copies_in_flight: int = 8) -> dict:
    """Run every job through the continuous-batching loop.  Jobs must be
    sorted by arrival time.  Returns latency and throughput statistics;
    per-job timestamps are written into the JobState objects.

    At most ``max_copies_in_flight`` host-to-device copies are queued at a
    time: a deep copy queue can block the host thread inside the runtime,
    and while it is blocked no transform or device-to-host copy is issued,
    so the two directions of the host link would run one after the other
    instead of together."""
    arena = Arena(arena_samples)
    n = len(jobs)
    nxt = 0
    pending: deque = deque()
    # copies complete in issue order on their streams: only the head of
    # each queue needs polling
    copying: deque = deque()
    ready: List[JobState] = []
    returning: deque = deque()
    finished = 0
    rejected = 0
    launch_id = 0
    peak_used = 0
    while finished + rejected < n:
        t = executor.now()
        while nxt < n and jobs[nxt].arrival_s <= t:
            pending.append(jobs[nxt])
            nxt += 1
        progressed = False
        # admission: arrival order, while the head of the queue fits
        while pending and len(copying) < max_copies_in_flight:
            head = pending[0]
            if not arena.fits_ever(head.samples) or head.samples > max_launch_samples:
                pending.popleft()
                head.status = "rejected"
                rejected += 1
                if not reject_oversized:
                    raise RejectedJob("job %d needs %d samples" % (head.index, head.samples))
                progressed = True
                continue
            off = arena.alloc(head.samples)
            if off is None:
                break
            pending.popleft()
            head.off = off
            head.admitted_s = t
            head.status = "copying"
            head.tokens["in"] = executor.h2d(head)
            copying.append(head)
            peak_used = max(peak_used, arena.used)
            progressed = True
            # A lone job on an idle device goes to the transform stream at
            # once, behind its own copy (the stream waits for the copy on
            # the device): at light load it pays no host round trip between
            # copy and transform, and its work list is compiled while the
            # copy runs.  Jobs that arrive meanwhile wait for the next
            # launch, as they would have anyway.
            if len(copying) == 1 and not ready and not pending and executor.stream_idle():
                j = copying.popleft()
                tok = executor.compute([j], after=j.tokens["in"])
                j.status = "computing"
                j.launch = launch_id
                j.tokens["comp"] = tok
                j.tokens["out"] = executor.d2h(j, tok)
                returning.append(j)
                launch_id += 1
        # inputs that have landed
        while copying and executor.done(copying[0].tokens["in"]):
            j = copying.popleft()
            j.status = "ready"
            ready.append(j)
            progressed = True
        # pack every ready job into one launch when the transform stream is free
        if ready and executor.stream_idle():
            batch, total = [], 0
            rest = []
            for j in ready:
                if total + j.samples <= max_launch_samples:
                    batch.append(j)
                    total += j.samples
                else:
                    rest.append(j)
            tok = executor.compute(batch)
            for j in batch:
                j.status = "computing"
                j.launch = launch_id
                j.tokens["comp"] = tok
                j.tokens["out"] = executor.d2h(j, tok)
                returning.append(j)
            launch_id += 1
            ready = rest
            progressed = True
        # spectra back on the host: release the arena
        while returning and executor.done(returning[0].tokens["out"]):
            j = returning.popleft()
            j.status = "done"
            j.done_s = executor.now()
            arena.release(j.off, j.samples)
            finished += 1
            progressed = True
        if not progressed:
            until = jobs[nxt].arrival_s if nxt < n else math.inf
            executor.advance(until)
    if hasattr(executor, "finish"):
        executor.finish()
    return summarize(jobs, launch_id, peak_used)


def summarize(jobs: List[JobState], launches: int = 0, peak_used: int = 0) -> dict:
    import numpy as np
    done = [j for j in jobs if j.status == "done"]
    lat = np.array([j.done_s - j.arrival_s for j in done]) if done else np.zeros(1)
    span = (max(j.done_s for j in done) - min(j.arrival_s for j in jobs)) if done else 0.0
    samples = sum(j.samples for j in done)
    return {
        "jobs": len(jobs), "completed": len(done),
        "rejected": sum(j.status == "rejected" for j in jobs),
        "launches": launches, "makespan_s": span,
        "jobs_per_s": len(done) / span if span > 0 else 0.0,
        "samples_per_s": samples / span if span > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "peak_arena_samples": peak_used,
    }


def serve_fifo(jobs: List[JobState], plans: dict, arena, stream=None) -> dict:
    """The plain batched path as the reference: one job at a time, copy in,
    one fft_exec_segments over the job's segments, copy out, wait.  ``plans``
    maps seg_len -> Plan with batch >= the largest job; ``arena`` is a
    complex64 device tensor holding the largest job."""
    import ctypes
    import torch
    hip = _hip()
    t0 = time.perf_counter()
    sh = torch.cuda.current_stream().cuda_stream if stream is None else stream
    base = arena.data_ptr()
    for j in jobs:
        while time.perf_counter() - t0 < j.arrival_s:
            time.sleep(20e-6)
        nb = j.samples * SAMPLE_BYTES
        rc = hip.hipMemcpyAsync(ctypes.c_void_p(base), ctypes.c_void_p(j.host_in),
                                ctypes.c_size_t(nb), 1, ctypes.c_void_p(sh))
        assert rc == 0
        plans[j.seg_len].exec_ptr(base, base, sh, batch=j.n_seg)
        rc = hip.hipMemcpyAsync(ctypes.c_void_p(j.host_out), ctypes.c_void_p(base),
                                ctypes.c_size_t(nb), 2, ctypes.c_void_p(sh))
        assert rc == 0
        torch.cuda.synchronize()
        j.done_s = time.perf_counter() - t0
        j.status = "done"
    return summarize(jobs, len(jobs), 0)
