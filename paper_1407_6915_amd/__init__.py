"""Batched segment FFT on AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libfftseg.so`` (C ABI in ``include/fftseg.h``):
argument marshalling only -- every step of the transform runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.

The method (Tsiomenko & Rees, arXiv:1407.6915, Sec. III): a long signal is
cut into fixed-length segments, each an <offset, FFT segment> record; one
batched plan transforms all segments of a block, and each spectrum is kept
at its record's offset.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import List, Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfftseg.so")

FORWARD = -1
INVERSE = +1

STATUS = {
    0: "FFT_OK",
    -1: "FFT_ERR_INVALID_ARG",
    -2: "FFT_ERR_UNSUPPORTED_LENGTH",
    -3: "FFT_ERR_OUT_OF_MEMORY",
    -4: "FFT_ERR_ALIGNMENT",
    -5: "FFT_ERR_OVERLAP",
    -6: "FFT_ERR_HIP",
    -7: "FFT_ERR_CALLBACK",
    -8: "FFT_ERR_BOUNDS",
    -9: "FFT_ERR_TIMEOUT",
}


class FFTError(RuntimeError):
    """A library call failed; ``status`` is the fft_status_t value."""

    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.name, message))


class StreamStats(ctypes.Structure):
    """fft_stream_stats_t: wall/callback/copy/transform seconds and bytes."""
    _fields_ = [("wall_s", ctypes.c_double), ("fill_s", ctypes.c_double),
                ("drain_s", ctypes.c_double), ("h2d_s", ctypes.c_double),
                ("d2h_s", ctypes.c_double), ("compute_s", ctypes.c_double),
                ("bytes_h2d", ctypes.c_uint64), ("bytes_d2h", ctypes.c_uint64),
                ("chunks_done", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


FILL_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                           ctypes.c_void_p, ctypes.c_uint64)
DRAIN_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                            ctypes.c_void_p, ctypes.c_uint64)

class ChunkTimes(ctypes.Structure):
    """fft_chunk_times_t: one chunk's copy-in, transform and copy-out
    intervals on the GPU clock (ms from chunk 0's copy-in start)."""
    _fields_ = [("chunk", ctypes.c_uint64),
                ("h2d_start_ms", ctypes.c_float), ("h2d_end_ms", ctypes.c_float),
                ("compute_start_ms", ctypes.c_float), ("compute_end_ms", ctypes.c_float),
                ("d2h_start_ms", ctypes.c_float), ("d2h_end_ms", ctypes.c_float)]


class WorkItem(ctypes.Structure):
    """fft_work_t: sample offsets of one segment and of its spectrum."""
    _fields_ = [("in_off", ctypes.c_uint64), ("out_off", ctypes.c_uint64),
                ("segment_len", ctypes.c_uint32), ("job", ctypes.c_uint32)]


_lib = None


def build() -> str:
    """Compile libfftseg.so for gfx950 in-tree (hipcc)."""
    from . import _build
    global _lib
    _lib = None
    return _build.build()


def _sig(lib, name, restype, argtypes):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = argtypes


def lib():
    """The loaded library (built first if no build exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    # torch ships its own copy of the HIP runtime: load it first so that this
    # library binds to the same copy (one HIP runtime per process; a second
    # copy loaded later cannot open the GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint64
    _sig(L, "fft_plan_create", vp, [sz, sz, i32])
    _sig(L, "fft_plan_create_variant", vp, [sz, sz, i32, i32])
    _sig(L, "fft_plan_create_real", vp, [sz, sz, i32])
    _sig(L, "fft_variant_count", i32, [sz])
    _sig(L, "fft_split_info", i32, [sz, ctypes.POINTER(sz), ctypes.POINTER(sz),
                                    ctypes.POINTER(i32), ctypes.POINTER(i32)])
    _sig(L, "fft_plan_create_split", vp, [sz, sz, i32, i32, i32])
    _sig(L, "fft_exec_segments", i32, [vp, vp, vp, vp])
    _sig(L, "fft_exec_segments_n", i32, [vp, vp, vp, sz, vp])
    _sig(L, "fft_exec_segments_noalloc", i32, [sz, sz, i32, vp, vp, vp])
    _sig(L, "fft_plan_destroy", i32, [vp])
    _sig(L, "fft_last_status", i32, [])
    _sig(L, "fft_last_error", ctypes.c_char_p, [])
    _sig(L, "fft_plan_factorize", i32, [sz, ctypes.POINTER(i32), i32])
    _sig(L, "fft_plan_describe", i32, [vp, ctypes.c_char_p, sz])
    _sig(L, "fft_plan_scratch_bytes", sz, [vp])
    _sig(L, "fft_exec_stream", i32, [vp, u64, FILL_FN, DRAIN_FN, vp, i32,
                                     ctypes.POINTER(u64), ctypes.POINTER(StreamStats)])
    _sig(L, "fft_exec_stream_pinned", i32, [vp, u64, ctypes.POINTER(vp), i32,
                                            ctypes.POINTER(vp), i32, i32,
                                            ctypes.POINTER(StreamStats)])
    _sig(L, "fft_stream_last_timeline", i32, [vp, ctypes.POINTER(ChunkTimes), sz])
    _sig(L, "fft_host_alloc", vp, [sz])
    _sig(L, "fft_host_free", i32, [vp])
    _sig(L, "fft_exec_file", i32, [vp, ctypes.c_char_p, u64, ctypes.c_char_p, u64, u64, u64,
                                   i32, i32, ctypes.POINTER(u64), ctypes.POINTER(StreamStats)])
    _sig(L, "fft_exec_frames", i32, [vp, vp, sz, vp, sz, sz, vp, vp])
    _sig(L, "fft_worklist_supported", i32, [ctypes.c_uint32])
    _sig(L, "fft_worklist_indexed_count", i32, [ctypes.c_uint32])
    _sig(L, "fft_worklist_create", vp, [ctypes.POINTER(WorkItem), sz, i32])
    _sig(L, "fft_worklist_reset", i32, [vp, ctypes.POINTER(WorkItem), sz, vp])
    _sig(L, "fft_worklist_exec", i32, [vp, vp, vp, vp])
    _sig(L, "fft_worklist_exec_graph", i32, [vp, vp, vp, vp])
    _sig(L, "fft_exec_worklist", i32, [ctypes.POINTER(WorkItem), sz, i32, vp, vp, vp])
    _sig(L, "fft_worklist_cache_clear", i32, [])
    _sig(L, "fft_worklist_status", i32, [vp, vp])
    _sig(L, "fft_worklist_describe", i32, [vp, ctypes.c_char_p, sz])
    _sig(L, "fft_worklist_destroy", i32, [vp])
    _sig(L, "fft_exec_segments_graph", i32, [vp, vp, vp, vp])
    _sig(L, "fft_autotune", i32, [sz, sz, i32, ctypes.c_char_p,
                                  ctypes.POINTER(ctypes.c_double)])
    _sig(L, "fft_tune_load", i32, [ctypes.c_char_p])
    _sig(L, "fft_tune_clear", i32, [])
    _lib = L
    return L


def last_error() -> str:
    return lib().fft_last_error().decode(errors="replace")


def _check(status: int) -> int:
    if status < 0:
        raise FFTError(status, last_error())
    return status


def factorize(n: int) -> List[int]:
    """Radices the planner uses for one pass of length n."""
    buf = (ctypes.c_int * 32)()
    k = _check(lib().fft_plan_factorize(n, buf, 32))
    return [buf[i] for i in range(k)]


def variant_count(n: int) -> int:
    """Single-pass kernel variants compiled in for length n."""
    return int(lib().fft_variant_count(n))


def split_info(n: int):
    """(n1, n2, column variants, row variants) of a two-pass length, or None."""
    n1, n2 = ctypes.c_size_t(), ctypes.c_size_t()
    c, r = ctypes.c_int(), ctypes.c_int()
    ok = lib().fft_split_info(n, ctypes.byref(n1), ctypes.byref(n2), ctypes.byref(c),
                              ctypes.byref(r))
    return (n1.value, n2.value, c.value, r.value) if ok == 1 else None


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tensor_ptr(t, n_samples: int, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != torch.complex64:
        raise TypeError("%s must be complex64 (got %s)" % (name, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be on a GPU" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < n_samples:
        raise ValueError("%s holds %d samples, %d needed" % (name, t.numel(), n_samples))
    return t.data_ptr()


class Plan:
    """Plan for ``batch`` segments of ``segment_len`` complex64 samples.

    ``exec(x, out)`` maps the record at byte offset s*N*8 of x to its
    spectrum at the same offset of out (in place when out is x).
    """

    def __init__(self, segment_len: int, batch: int, direction: int = FORWARD,
                 variant: Optional[int] = None, split_variants=None):
        L = lib()
        if split_variants is not None:
            h = L.fft_plan_create_split(segment_len, batch, direction, split_variants[0],
                                        split_variants[1])
        elif variant is None:
            h = L.fft_plan_create(segment_len, batch, direction)
        else:
            h = L.fft_plan_create_variant(segment_len, batch, direction, variant)
        if not h:
            raise FFTError(L.fft_last_status(), last_error())
        self._h = h
        self.segment_len = segment_len
        self.batch = batch
        self.direction = direction

    @property
    def handle(self) -> int:
        if not self._h:
            raise ValueError("plan is destroyed")
        return self._h

    def exec_ptr(self, in_ptr: int, out_ptr: int, stream: int = 0,
                 batch: Optional[int] = None) -> None:
        """Raw device pointers (the C call, argument checks included)."""
        if batch is None:
            _check(lib().fft_exec_segments(self.handle, in_ptr, out_ptr, stream))
        else:
            _check(lib().fft_exec_segments_n(self.handle, in_ptr, out_ptr, batch,
                                             stream))

    def exec_graph_ptr(self, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
        """fft_exec_segments through a captured hipGraph."""
        _check(lib().fft_exec_segments_graph(self.handle, in_ptr, out_ptr, stream))

    def exec(self, x, out=None, stream=None, batch: Optional[int] = None):
        """Transform torch complex64 GPU tensors; returns ``out``."""
        import torch
        b = self.batch if batch is None else batch
        n = b * self.segment_len
        ip = _tensor_ptr(x, n, "x")
        if out is None:
            out = torch.empty(n, dtype=torch.complex64, device=x.device)
        op = _tensor_ptr(out, n, "out")
        self.exec_ptr(ip, op, _stream_handle(stream), batch)
        return out

    def exec_frames_ptr(self, in_ptr: int, in_len: int, out_ptr: int, n_frames: int,
                        hop: int, window_ptr: int = 0, stream: int = 0) -> None:
        """fft_exec_frames on raw device pointers."""
        _check(lib().fft_exec_frames(self.handle, in_ptr, in_len, out_ptr, n_frames, hop,
                                     window_ptr or None, stream))

    def exec_frames(self, x, hop: int, n_frames: Optional[int] = None, window=None,
                    out=None, stream=None):
        """Short-time transform: frame s starts at sample s*hop of the
        complex64 GPU tensor x and is multiplied by ``window`` (a float32
        GPU tensor of segment_len values, or None) before its transform.
        n_frames defaults to every whole frame x holds, capped at the
        plan's batch.  Returns ``out`` ([n_frames * segment_len])."""
        import torch
        n = self.segment_len
        total = x.numel()
        if n_frames is None:
            n_frames = min(self.batch, (total - n) // hop + 1 if total >= n else 0)
        ip = _tensor_ptr(x, 0, "x")
        wp = 0
        if window is not None:
            if window.dtype != torch.float32 or not window.is_cuda or not window.is_contiguous():
                raise TypeError("window must be a contiguous float32 GPU tensor")
            if window.numel() != n:
                raise ValueError("window holds %d values, %d needed" % (window.numel(), n))
            wp = window.data_ptr()
        if out is None:
            out = torch.empty(max(n_frames, 0) * n, dtype=torch.complex64, device=x.device)
        op = _tensor_ptr(out, n_frames * n, "out")
        self.exec_frames_ptr(ip, total, op, n_frames, hop, wp, _stream_handle(stream))
        return out

    def exec_stream(self, n_chunks: int, fill, drain=None, n_slots: int = 3):
        """Stream n_chunks chunks of this plan's batch through the GPU.

        ``fill``/``drain`` are either Python callables ``f(chunk, ptr,
        nbytes) -> int`` (0 = success) working on the library's pinned slot
        at host address ptr, or ``(address, user)`` pairs naming a native C
        callback and the object whose address it receives.  Returns
        (status, failed_chunk or None, stats dict); a callback failure is
        reported in the status, not raised.
        """
        user = None
        keep = []

        def wrap(cb, ftype):
            nonlocal user
            if cb is None:
                return ftype()
            if isinstance(cb, tuple):
                addr, obj = cb
                if user is not None and obj is not user:
                    raise ValueError("native fill and drain must share one user object")
                user = obj
                return ftype(addr)
            f = ftype(lambda _u, c, ptr, nb: int(cb(int(c), ptr, int(nb))))
            keep.append(f)
            return f

        f_fill = wrap(fill, FILL_FN)
        f_drain = wrap(drain, DRAIN_FN)
        uptr = ctypes.cast(ctypes.pointer(user), ctypes.c_void_p) if user is not None else None
        failed = ctypes.c_uint64(0)
        st = StreamStats()
        rc = lib().fft_exec_stream(self.handle, n_chunks, f_fill, f_drain, uptr,
                                   n_slots, ctypes.byref(failed), ctypes.byref(st))
        if rc < 0 and rc != -7:
            raise FFTError(rc, last_error())
        fc = None if failed.value == 2 ** 64 - 1 else int(failed.value)
        return rc, fc, st.as_dict()

    def exec_file(self, in_path: str, out_path: str, n_chunks: int, first_chunk: int = 0,
                  in_offset: int = 0, out_offset: int = 0, n_slots: int = 3,
                  io_threads: int = 8):
        """Stream chunks of a signal file through the GPU, spectra written
        at the same relative offsets of out_path.  Returns (status,
        failed_chunk or None, stats); an I/O failure is reported in the
        status, other errors raise."""
        failed = ctypes.c_uint64(0)
        st = StreamStats()
        rc = lib().fft_exec_file(self.handle, in_path.encode(), in_offset, out_path.encode(),
                                 out_offset, first_chunk, n_chunks, n_slots, io_threads,
                                 ctypes.byref(failed), ctypes.byref(st))
        if rc < 0 and rc != -7:
            raise FFTError(rc, last_error())
        fc = None if failed.value == 2 ** 64 - 1 else int(failed.value)
        return rc, fc, st.as_dict()

    def exec_stream_pinned(self, n_chunks: int, host_in, host_out, n_slots: int = 3):
        """Stream through caller-owned pinned host buffers (lists of host
        addresses): chunk c reads host_in[c % len] and writes host_out[c % len]."""
        vin = (ctypes.c_void_p * len(host_in))(*host_in)
        vout = (ctypes.c_void_p * len(host_out))(*host_out)
        st = StreamStats()
        _check(lib().fft_exec_stream_pinned(self.handle, n_chunks, vin, len(host_in),
                                            vout, len(host_out), n_slots,
                                            ctypes.byref(st)))
        return st.as_dict()

    def stream_timeline(self) -> List[dict]:
        """Per-chunk copy and transform intervals of the last streamed call
        (ms on the GPU clock from chunk 0's copy-in start)."""
        L = lib()
        n = _check(L.fft_stream_last_timeline(self.handle, None, 0))
        arr = (ChunkTimes * max(n, 1))()
        _check(L.fft_stream_last_timeline(self.handle, arr, n))
        return [{f: getattr(arr[i], f) for f, _ in ChunkTimes._fields_} for i in range(n)]

    def describe(self) -> dict:
        L = lib()
        need = _check(L.fft_plan_describe(self.handle, None, 0))
        buf = ctypes.create_string_buffer(need + 1)
        _check(L.fft_plan_describe(self.handle, buf, need + 1))
        return json.loads(buf.value.decode())

    @property
    def scratch_bytes(self) -> int:
        return int(lib().fft_plan_scratch_bytes(self.handle))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().fft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def exec_segments_noalloc_ptr(segment_len: int, batch: int, in_ptr: int, out_ptr: int,
                              direction: int = FORWARD, stream: int = 0) -> None:
    """fft_exec_segments_noalloc: the batched transform without a plan or
    any device allocation (tables and scratch in the library's static
    device array; calls overlapping on one GPU race)."""
    _check(lib().fft_exec_segments_noalloc(segment_len, batch, direction, in_ptr, out_ptr,
                                           stream))


class RealPlan(Plan):
    """Plan for ``batch`` real segments of even length ``segment_len``.

    Forward: float32 [batch * N] -> complex64 [batch * (N/2+1)] (bins
    0..N/2 of every segment).  Inverse: complex64 bins -> float32 samples,
    unnormalised.  Always out of place.
    """

    def __init__(self, segment_len: int, batch: int, direction: int = FORWARD):
        L = lib()
        h = L.fft_plan_create_real(segment_len, batch, direction)
        if not h:
            raise FFTError(L.fft_last_status(), last_error())
        self._h = h
        self.segment_len = segment_len
        self.batch = batch
        self.direction = direction

    @property
    def bins(self) -> int:
        return self.segment_len // 2 + 1

    def exec(self, x, out=None, stream=None, batch: Optional[int] = None):
        import torch
        b = self.batch if batch is None else batch
        real_n, cplx_n = b * self.segment_len, b * self.bins
        if self.direction == FORWARD:
            in_dt, out_dt, need_in, need_out = torch.float32, torch.complex64, real_n, cplx_n
        else:
            in_dt, out_dt, need_in, need_out = torch.complex64, torch.float32, cplx_n, real_n
        for t, dt, need, name in ((x, in_dt, need_in, "x"), (out, out_dt, need_out, "out")):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or t.dtype != dt:
                raise TypeError("%s must be a %s tensor" % (name, dt))
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("%s must be a contiguous GPU tensor" % name)
            if t.numel() < need:
                raise ValueError("%s holds %d values, %d needed" % (name, t.numel(), need))
        if out is None:
            out = torch.empty(need_out, dtype=out_dt, device=x.device)
        self.exec_ptr(x.data_ptr(), out.data_ptr(), _stream_handle(stream), batch)
        return out


class WorkList:
    """Segments of uneven length at arbitrary sample offsets, run by one
    persistent kernel launch.  ``entries`` is a sequence of
    (in_off, out_off, segment_len[, job]) in samples, or a numpy structured
    array with those fields."""

    @staticmethod
    def _items(entries):
        import numpy as np
        work_dtype = np.dtype([("in_off", "<u8"), ("out_off", "<u8"),
                               ("segment_len", "<u4"), ("job", "<u4")])
        if (isinstance(entries, np.ndarray) and entries.dtype == work_dtype
                and entries.ndim == 1 and entries.flags["C_CONTIGUOUS"] and len(entries)):
            # same layout as fft_work_t: hand the array over without a copy
            # (the caller's array must stay alive for the call)
            return entries.ctypes.data_as(ctypes.POINTER(WorkItem)), len(entries)
        if isinstance(entries, np.ndarray) and entries.dtype.names:
            arr = np.ascontiguousarray(entries)
            n = len(arr)
            items = (WorkItem * max(n, 1))()
            buf = np.frombuffer(items, dtype=np.dtype([("in_off", "<u8"), ("out_off", "<u8"),
                                                       ("segment_len", "<u4"), ("job", "<u4")]))[:n]
            for f in ("in_off", "out_off", "segment_len"):
                buf[f] = arr[f]
            buf["job"] = arr["job"] if "job" in arr.dtype.names else 0
        else:
            entries = list(entries)
            n = len(entries)
            items = (WorkItem * max(n, 1))()
            for i, e in enumerate(entries):
                items[i].in_off, items[i].out_off, items[i].segment_len = e[0], e[1], e[2]
                items[i].job = e[3] if len(e) > 3 else 0
        return items, n

    def __init__(self, entries=(), direction: int = FORWARD):
        items, n = self._items(entries)
        L = lib()
        h = L.fft_worklist_create(items, n, direction)
        if not h:
            raise FFTError(L.fft_last_status(), last_error())
        self._h = h
        self.n_items = n
        self.direction = direction

    @property
    def handle(self) -> int:
        if not self._h:
            raise ValueError("work list is destroyed")
        return self._h

    def reset(self, entries, stream=None) -> None:
        """Replace the entries (upload ordered on ``stream``)."""
        items, n = self._items(entries)
        _check(lib().fft_worklist_reset(self.handle, items, n, _stream_handle(stream)))
        self.n_items = n

    def exec_ptr(self, in_base: int, out_base: int, stream: int = 0, graph: bool = False):
        f = lib().fft_worklist_exec_graph if graph else lib().fft_worklist_exec
        _check(f(self.handle, in_base, out_base, stream))

    def exec(self, x, out, stream=None, graph: bool = False):
        """Run on torch complex64 GPU tensors holding every entry's range."""
        ip = _tensor_ptr(x, 0, "x")
        op = _tensor_ptr(out, 0, "out")
        self.exec_ptr(ip, op, _stream_handle(stream), graph)
        return out

    def status(self, stream=None) -> None:
        """Synchronise and raise FFTError if the last run did not complete."""
        _check(lib().fft_worklist_status(self.handle, _stream_handle(stream)))

    def stream_timeline(self) -> List[dict]:
        """Per-chunk copy and transform intervals of the last streamed call
        (ms on the GPU clock from chunk 0's copy-in start)."""
        L = lib()
        n = _check(L.fft_stream_last_timeline(self.handle, None, 0))
        arr = (ChunkTimes * max(n, 1))()
        _check(L.fft_stream_last_timeline(self.handle, arr, n))
        return [{f: getattr(arr[i], f) for f, _ in ChunkTimes._fields_} for i in range(n)]

    def describe(self) -> dict:
        L = lib()
        need = _check(L.fft_worklist_describe(self.handle, None, 0))
        buf = ctypes.create_string_buffer(need + 1)
        _check(L.fft_worklist_describe(self.handle, buf, need + 1))
        return json.loads(buf.value.decode())

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().fft_worklist_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def exec_worklist_ptr(entries, in_base: int, out_base: int, direction: int = FORWARD,
                      stream: int = 0) -> None:
    """One call per uneven batch (fft_exec_worklist): ``entries`` as for
    WorkList, raw device base pointers."""
    items, n = WorkList._items(entries)
    _check(lib().fft_exec_worklist(items, n, direction, in_base, out_base, stream))


def exec_worklist(entries, x, out, direction: int = FORWARD, stream=None):
    """fft_exec_worklist on torch complex64 GPU tensors holding every
    entry's range; returns ``out``."""
    exec_worklist_ptr(entries, _tensor_ptr(x, 0, "x"), _tensor_ptr(out, 0, "out"), direction,
                      _stream_handle(stream))
    return out


def worklist_cache_clear() -> None:
    """Free the work lists kept by fft_exec_worklist."""
    _check(lib().fft_worklist_cache_clear())


def worklist_supported(n: int) -> bool:
    return bool(lib().fft_worklist_supported(n))


def indexed_count(n: int) -> int:
    """Indexed one-pass kernels a work list can route length n through."""
    return int(lib().fft_worklist_indexed_count(n))


def autotune(segment_len: int, batch: int, direction: int = FORWARD,
             path: Optional[str] = None):
    """Time every variant x grid size; returns (configurations timed, best us)."""
    best = ctypes.c_double(0.0)
    k = _check(lib().fft_autotune(segment_len, batch, direction,
                                  path.encode() if path else None, ctypes.byref(best)))
    return k, best.value


def tune_load(path: str) -> int:
    return _check(lib().fft_tune_load(path.encode()))


def tune_clear() -> None:
    _check(lib().fft_tune_clear())


class HostBuffer:
    """Pinned host memory from fft_host_alloc, freed by close() (or the
    context manager); ``ptr`` is its address."""

    def __init__(self, nbytes: int):
        p = lib().fft_host_alloc(nbytes)
        if not p:
            raise FFTError(lib().fft_last_status(), last_error())
        self.ptr = int(p)
        self.nbytes = int(nbytes)

    def view(self, dtype="complex64"):
        """numpy view of the buffer (valid until close)."""
        import numpy as np
        buf = (ctypes.c_char * self.nbytes).from_address(self.ptr)
        return np.frombuffer(buf, dtype=dtype)

    def close(self) -> None:
        if getattr(self, "ptr", 0):
            _check(lib().fft_host_free(self.ptr))
            self.ptr = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
