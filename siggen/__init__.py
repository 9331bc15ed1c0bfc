"""Seeded synthetic input generators shared by the oracle tests and the GPU
library's tests and benchmark.

This package holds no FFT arithmetic: it draws Philox4x32-10 random numbers
and synthesises signals (Gaussian noise, bin-centred tones, a per-segment
linear chirp) sample by sample from a global sample index, so any segment or
chunk can be regenerated alone.  ``siggen.c`` is the implementation;
``workloads`` holds the recipes of the five benchmark workloads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "siggen.c")
_LIB_PATH = os.path.join(_HERE, "libsiggen.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``siggen.c`` with gcc (-O3, OpenMP, no floating-point
    contraction, so that every instruction-set clone gives the same bits)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
           "-fno-fast-math", "-ffp-contract=off", "-fno-math-errno",
           "-fno-trapping-math",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CSignal(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_uint32),
        ("n_tones", ctypes.c_uint32),
        ("sigma", ctypes.c_double),
        ("seg_len", ctypes.c_uint64),
        ("tone_bin", ctypes.POINTER(ctypes.c_int64)),
        ("tone_amp", ctypes.POINTER(ctypes.c_double)),
        ("tone_phase", ctypes.POINTER(ctypes.c_double)),
        ("chirp_amp", ctypes.c_double),
    ]


class _CChunkSource(ctypes.Structure):
    _fields_ = [
        ("sig", _CSignal),
        ("first_sample", ctypes.c_uint64),
        ("chunk_samples", ctypes.c_uint64),
        ("threads", ctypes.c_int),
        ("check_seg_len", ctypes.c_uint64),
        ("n_chunks", ctypes.c_uint64),
        ("energy_in", ctypes.c_void_p),
        ("energy_out", ctypes.c_void_p),
        ("saved_out", ctypes.c_void_p),
        ("drain_threads", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.sg_philox4x32_10.restype = None
    lib.sg_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
    lib.sg_fill.restype = ctypes.c_int
    lib.sg_fill.argtypes = [ctypes.POINTER(_CSignal), ctypes.c_uint64,
                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int]
    for name in ("sg_uniform", "sg_normal"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                      ctypes.c_uint64, ctypes.c_void_p]
    lib.sg_fill_segments.restype = ctypes.c_int
    lib.sg_fill_segments.argtypes = [ctypes.POINTER(_CSignal), ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int]
    lib.sg_energy.restype = ctypes.c_int
    lib.sg_energy.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_void_p, ctypes.c_int]
    for name in ("sg_fill_chunk", "sg_drain_chunk"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                      ctypes.c_uint64]
    lib.sg_set_isa.restype = ctypes.c_int
    lib.sg_set_isa.argtypes = [ctypes.c_int]
    lib.sg_test_ln.restype = ctypes.c_double
    lib.sg_test_ln.argtypes = [ctypes.c_double]
    lib.sg_test_turn.restype = None
    lib.sg_test_turn.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
    _lib = lib
    return lib


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, ...]:
    """One Philox4x32-10 block: 4 x uint32 counter, 2 x uint32 key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    _load().sg_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def uniform(seed: int, stream: int, first: int, count: int) -> np.ndarray:
    """``count`` uniform doubles in (0, 1) (53-bit) for draw indices
    first..first+count-1 of (seed, stream)."""
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().sg_uniform(seed, stream, first, count, out.ctypes.data)
    return out


def normal(seed: int, stream: int, first: int, count: int) -> np.ndarray:
    """``count`` standard normal doubles for draw indices first.. of
    (seed, stream)."""
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().sg_normal(seed, stream, first, count, out.ctypes.data)
    return out


@dataclass
class Signal:
    """A seeded synthetic complex signal cut into ``seg_len``-sample
    segments.  Sample g = noise(g) + tones(g mod seg_len) + chirp(g mod
    seg_len); see ``siggen.c`` for the exact definition."""
    seed: int
    seg_len: int
    sigma: float = 1.0
    stream: int = 0
    tones: List[Tuple[int, float, float]] = field(default_factory=list)
    chirp_amp: float = 0.0

    def _c(self):
        n = len(self.tones)
        bins = (ctypes.c_int64 * max(n, 1))(*[int(t[0]) for t in self.tones])
        amps = (ctypes.c_double * max(n, 1))(*[float(t[1]) for t in self.tones])
        phs = (ctypes.c_double * max(n, 1))(*[float(t[2]) for t in self.tones])
        cs = _CSignal(self.seed & 0xFFFFFFFFFFFFFFFF, self.stream & 0xFFFFFFFF,
                      n, float(self.sigma), int(self.seg_len),
                      ctypes.cast(bins, ctypes.POINTER(ctypes.c_int64)),
                      ctypes.cast(amps, ctypes.POINTER(ctypes.c_double)),
                      ctypes.cast(phs, ctypes.POINTER(ctypes.c_double)),
                      float(self.chirp_amp))
        return cs, (bins, amps, phs)

    def fill_ptr(self, first: int, count: int, ptr: int, threads: int = 0):
        """Write samples first..first+count-1 as interleaved float32 pairs
        to host address ``ptr`` (e.g. pinned memory)."""
        cs, keep = self._c()
        rc = _load().sg_fill(ctypes.byref(cs), first, count, ptr, threads)
        del keep
        if rc != 0:
            raise RuntimeError("sg_fill failed (%d)" % rc)

    def samples(self, first: int, count: int, threads: int = 0) -> np.ndarray:
        """Samples first..first+count-1 as a complex64 array."""
        out = np.empty(count, dtype=np.complex64)
        if count:
            self.fill_ptr(first, count, out.ctypes.data, threads)
        return out

    def segments(self, first_seg: int, n_seg: int, threads: int = 0) -> np.ndarray:
        """Segments first_seg..first_seg+n_seg-1 as complex64 [n_seg, seg_len]."""
        n = self.seg_len
        return self.samples(first_seg * n, n_seg * n, threads).reshape(n_seg, n)

    def segments_with_energy(self, first_seg: int, n_seg: int, threads: int = 0):
        """(segments as complex64 [n_seg, seg_len], each segment's energy
        sum |x|^2 of the stored float32 values in float64)."""
        n = self.seg_len
        out = np.empty((n_seg, n), dtype=np.complex64)
        e = np.empty(n_seg, dtype=np.float64)
        if n_seg:
            cs, keep = self._c()
            rc = _load().sg_fill_segments(ctypes.byref(cs), first_seg, n_seg,
                                          out.ctypes.data, e.ctypes.data, threads)
            del keep
            if rc != 0:
                raise RuntimeError("sg_fill_segments failed (%d)" % rc)
        return out, e

    def chunk_source(self, first_sample: int, chunk_samples: int,
                     threads: int = 0):
        """(callback address, user struct) for a native chunk producer of
        signature int(void *user, uint64 chunk, void *dst, uint64 bytes)
        that writes chunk c = samples first_sample + c*chunk_samples .. .
        Keep the returned struct alive while the callback may run."""
        cs, keep = self._c()
        src = _CChunkSource(cs, first_sample, chunk_samples, threads)
        src._keep = keep  # arrays referenced by the struct
        addr = ctypes.cast(_load().sg_fill_chunk, ctypes.c_void_p).value
        return addr, src

    def checked_chunk_source(self, chunk_segments: int, n_chunks: int,
                             first_seg: int = 0, threads: int = 0, drain_threads: int = 0):
        """Producer and consumer for streaming n_chunks chunks of
        chunk_segments whole segments (chunk c = segments first_seg +
        c*chunk_segments ..).  The producer records every segment's input
        energy, the consumer every segment's output energy and a copy of the
        first and last segment of each chunk (its sums on drain_threads
        threads, <= 0: threads).  Returns (fill address, drain address,
        user struct, CheckedStream with the arrays)."""
        n = self.seg_len
        chk = CheckedStream(
            energy_in=np.zeros((n_chunks, chunk_segments), np.float64),
            energy_out=np.zeros((n_chunks, chunk_segments), np.float64),
            saved_out=np.zeros((n_chunks, 2, n), np.complex64))
        cs, keep = self._c()
        src = _CChunkSource(cs, first_seg * n, chunk_segments * n, threads, n,
                            n_chunks, chk.energy_in.ctypes.data,
                            chk.energy_out.ctypes.data, chk.saved_out.ctypes.data,
                            drain_threads)
        src._keep = (keep, chk)
        L = _load()
        fill = ctypes.cast(L.sg_fill_chunk, ctypes.c_void_p).value
        drain = ctypes.cast(L.sg_drain_chunk, ctypes.c_void_p).value
        return fill, drain, src, chk


@dataclass
class CheckedStream:
    """Per-segment energies ([chunk, segment]) of a checked streamed run and
    the first and last output segment of every chunk ([chunk, 2, seg_len])."""
    energy_in: np.ndarray
    energy_out: np.ndarray
    saved_out: np.ndarray


def segment_energy(x: np.ndarray, threads: int = 0) -> np.ndarray:
    """Energy sum |x|^2 in float64 of each row of a complex64 [n_seg, n]
    array."""
    a = np.ascontiguousarray(x, dtype=np.complex64)
    if a.ndim == 1:
        a = a[None]
    out = np.empty(a.shape[0], dtype=np.float64)
    if a.shape[0]:
        rc = _load().sg_energy(a.ctypes.data, a.shape[0], a.shape[1], out.ctypes.data,
                               threads)
        if rc != 0:
            raise RuntimeError("sg_energy failed (%d)" % rc)
    return out


def set_isa(cap: int) -> int:
    """Cap the generator's instruction-set version (0 baseline x86-64, 1
    AVX2 + FMA, 2 AVX-512); returns the version then in use.  Every version
    computes the same bits."""
    return int(_load().sg_set_isa(cap))


def _test_ln(x: float) -> float:
    """The generator's own natural log (for its tests)."""
    return float(_load().sg_test_ln(x))


def _test_turn(num: int, den: int):
    """The generator's own (cos, sin)(2 pi num / den) (for its tests)."""
    o = (ctypes.c_double * 2)()
    _load().sg_test_turn(num, den, o)
    return float(o[0]), float(o[1])


def distinct_bins(seed: int, stream: int, n: int, count: int) -> List[int]:
    """``count`` distinct integer bins in [0, n) drawn in order from
    uniform draws of (seed, stream); duplicates are skipped."""
    bins: List[int] = []
    i = 0
    while len(bins) < count:
        u = uniform(seed, stream, i, 64)
        i += 64
        for v in u:
            b = int(v * n)
            if b not in bins:
                bins.append(b)
                if len(bins) == count:
                    break
    return bins


from . import workloads  # noqa: E402,F401
