"""FP64 CPU oracle for batched segment DFTs.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never loads it, and this package never imports the GPU library:
the two share no code.  Inputs come from the seeded generators in
``siggen`` (which hold no FFT arithmetic) or from closed forms in the tests.

What is computed (paper Sec. I-II: Cooley-Tukey reaches exactly the DFT;
Sec. III: a signal is cut into consecutive fixed-length segments, each
transformed on its own, each kept as an <offset, segment> record whose
offset is the byte offset from the start of the signal):

    X_s[k] = sum_n x_s[n] * exp(d * 2*pi*i * n*k / N),  d = -1 forward,
                                                         d = +1 inverse,
    no normalisation.

``dft_direct`` (O(N^2)) and ``fft_recursive`` (radix 2/3/5 decimation in
time) are the two independent routines of ``oracle.c``.  Everything else
here is marshalling plus the error metric the parity bar is stated in.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FORWARD = -1
INVERSE = +1

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (-O2, OpenMP, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    for name in ("orc_dft_direct", "orc_fft_recursive"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                      ctypes.c_uint64, ctypes.c_int]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    _lib = lib
    return lib


def max_threads() -> int:
    """Host threads an OpenMP region of the oracle uses."""
    return int(_load().orc_max_threads())


def _as_segments(x, n):
    """Exact upcast of complex64/complex128 data to a C-contiguous
    complex128 [batch, n] array."""
    a = np.asarray(x)
    if a.dtype not in (np.complex64, np.complex128):
        raise TypeError("oracle input must be complex64 or complex128")
    a = np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)
    if n <= 0 or a.size % n:
        raise ValueError("input size %d is not a multiple of n=%d" % (a.size, n))
    return a.reshape(-1, n)


def _run(fname, x, n, direction):
    if direction not in (FORWARD, INVERSE):
        raise ValueError("direction must be -1 (forward) or +1 (inverse)")
    a = _as_segments(x, n)
    out = np.empty_like(a)
    rc = getattr(_load(), fname)(a.ctypes.data, out.ctypes.data,
                                 a.shape[0], n, direction)
    if rc != 0:
        raise RuntimeError("%s failed with status %d" % (fname, rc))
    return out


def dft_direct(x, n: int, direction: int = FORWARD) -> np.ndarray:
    """O(N^2) DFT of every length-n segment of x (definition written out)."""
    return _run("orc_dft_direct", x, n, direction)


def fft_recursive(x, n: int, direction: int = FORWARD) -> np.ndarray:
    """Recursive radix-2/3/5 Cooley-Tukey DFT of every length-n segment."""
    return _run("orc_fft_recursive", x, n, direction)


def rel_l2(y, x_ref) -> np.ndarray:
    """Per-segment relative L2 error ||y - x_ref|| / ||x_ref|| in FP64.

    A segment whose reference is exactly zero scores 0 if y is exactly zero
    there and +inf otherwise.
    """
    y = np.asarray(y).astype(np.complex128).reshape(np.shape(x_ref))
    r = np.asarray(x_ref, dtype=np.complex128)
    num = np.sqrt(np.sum(np.abs(y - r) ** 2, axis=-1))
    den = np.sqrt(np.sum(np.abs(r) ** 2, axis=-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(den > 0, num / np.where(den > 0, den, 1.0),
                     np.where(num == 0, 0.0, np.inf))
    return e


def tolerance(n: int) -> float:
    """Per-segment rel-L2 bar for an FP32 transform of length n:
    5e-7 * log2(n) (log2 real-valued for non powers of two).  Length 1 is
    an exact copy and gets the length-2 bar."""
    return 5e-7 * max(np.log2(n), 1.0)


# --- segment <-> record mapping (paper Sec. III) ---------------------------

def record_offset(segment: int, n: int, bytes_per_sample: int,
                  base: int = 0) -> int:
    """Byte offset of segment ``segment`` in a signal of length-n segments
    (Sec. III: offset counts bytes from the beginning of the file)."""
    return base + segment * n * bytes_per_sample


def record_count(file_bytes: int, n: int, bytes_per_sample: int) -> int:
    """Whole segments of n samples in a file of ``file_bytes`` bytes."""
    return file_bytes // (n * bytes_per_sample)


def block_count(file_bytes: int, block_bytes: int) -> int:
    """Blocks (one map task each in Sec. III) covering ``file_bytes``."""
    return -(-file_bytes // block_bytes)


# --- overlapping, windowed segments (future work named in Sec. VI) ----------

def frames(x, n: int, hop: int, n_frames: int, window=None) -> np.ndarray:
    """The n_frames segments of a signal that start every ``hop`` samples
    (hop < n: consecutive segments overlap), each multiplied sample by sample
    by a real ``window`` of length n (None: rectangular), in FP64:

        f_s[j] = x[s*hop + j] * w[j],   0 <= s < n_frames, 0 <= j < n.

    With hop == n and no window this is the disjoint cut of Sec. III."""
    x = np.asarray(x).reshape(-1).astype(np.complex128)
    if hop < 1 or n_frames < 1 or (n_frames - 1) * hop + n > x.size:
        raise ValueError("frames outside the signal")
    out = np.empty((n_frames, n), dtype=np.complex128)
    for s in range(n_frames):
        out[s] = x[s * hop:s * hop + n]
    if window is not None:
        w = np.asarray(window, dtype=np.float64).reshape(-1)
        if w.size != n:
            raise ValueError("window length must equal n")
        out *= w[None, :]
    return out


def short_time(x, n: int, hop: int, n_frames: int, window=None,
               direction: int = FORWARD) -> np.ndarray:
    """Spectra of ``frames(...)``: each frame transformed by the recursive
    FFT of this module."""
    return fft_recursive(frames(x, n, hop, n_frames, window), n, direction)


# --- real-input segments (Sec. III: float32 samples, 4 bytes each) ---------

def real_forward(x, n: int) -> np.ndarray:
    """Spectrum of every real length-n segment (n even), bins 0..n/2:

        X_s[k] = sum_n x_s[n] exp(-2 pi i n k / N),  0 <= k <= N/2,

    the remaining bins being conj(X_s[N-k]) for real input.  Computed as
    the complex DFT of the real samples (imaginary parts zero)."""
    a = np.asarray(x)
    if a.dtype not in (np.float32, np.float64):
        raise TypeError("real oracle input must be float32 or float64")
    if n < 2 or n % 2:
        raise ValueError("real segments need an even length")
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size % n:
        raise ValueError("input size %d is not a multiple of n=%d" % (a.size, n))
    full = fft_recursive(a.astype(np.complex128), n, FORWARD)
    return np.ascontiguousarray(full[:, :n // 2 + 1])


def real_inverse(spec, n: int) -> np.ndarray:
    """Real length-n segments from their bins 0..n/2, unnormalised:

        x_s[j] = sum_{k<N} X_s[k] exp(+2 pi i j k / N),  X_s[N-k] = conj X_s[k].

    Bins 0 and N/2 of a real signal are real; their imaginary parts are
    ignored (the real part of the inverse of the Hermitian extension)."""
    a = np.asarray(spec)
    if a.dtype not in (np.complex64, np.complex128):
        raise TypeError("spectrum must be complex64 or complex128")
    if n < 2 or n % 2:
        raise ValueError("real segments need an even length")
    h = n // 2 + 1
    a = np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)
    if a.size % h:
        raise ValueError("spectrum size %d is not a multiple of n/2+1=%d" % (a.size, h))
    a = a.reshape(-1, h)
    full = np.empty((a.shape[0], n), dtype=np.complex128)
    full[:, :h] = a
    full[:, h:] = np.conj(a[:, 1:n // 2][:, ::-1])
    return fft_recursive(full, n, INVERSE).real.copy()
