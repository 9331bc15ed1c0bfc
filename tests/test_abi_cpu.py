"""The C-ABI library on a host without a GPU: it loads, exports every
function include/*.h declares, and rejects bad arguments before touching
the device."""
import ctypes
import glob
import os
import re

import pytest

import paper_1407_6915_amd as fs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w \*]*?\b(fft_\w+)\s*\(", src, re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "fft_plan_create" in names and "fft_exec_segments" in names
    lib = ctypes.CDLL(fs.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("args,status", [
    ((0, 1, -1), "FFT_ERR_INVALID_ARG"),
    ((1024, 0, -1), "FFT_ERR_INVALID_ARG"),
    ((1024, 1, 0), "FFT_ERR_INVALID_ARG"),
    ((1024, 1, 2), "FFT_ERR_INVALID_ARG"),
    ((7, 1, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),
    ((1024 * 7, 1, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),
    ((1 << 25, 1, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),
    ((1024, 1 << 62, -1), "FFT_ERR_INVALID_ARG"),
])
def test_create_rejects_bad_arguments(args, status):
    with pytest.raises(fs.FFTError) as ei:
        fs.Plan(*args)
    assert ei.value.name == status
    assert fs.lib().fft_last_status() == ei.value.status
    assert fs.last_error()


def test_null_plan_calls():
    L = fs.lib()
    assert L.fft_plan_destroy(None) == 0
    assert L.fft_exec_segments(None, None, None, None) == -1
    assert L.fft_plan_describe(None, None, 0) == -1
    assert L.fft_plan_scratch_bytes(None) == 0


def test_host_alloc_argument_checks():
    L = fs.lib()
    assert not L.fft_host_alloc(0)
    assert L.fft_last_status() == -1 and fs.last_error()
    assert L.fft_host_free(None) == 0
    assert L.fft_stream_last_timeline(None, None, 0) == -1


def test_factorize_matches_lengths():
    for n in (2, 16, 256, 1000, 1024, 1536, 4096, 6000, 16384, 65536, 3 ** 9,
              2 * 3 * 5 * 7 * 0 + 30, 1 << 20):
        r = fs.factorize(n)
        p = 1
        for v in r:
            assert v in (2, 3, 4, 5, 6, 8, 10, 12, 15, 16, 20, 25, 32)
            p *= v
        assert p == n, (n, r)
    assert fs.factorize(4096) in ([16, 16, 16], [8, 8, 8, 8])
    with pytest.raises(fs.FFTError):
        fs.factorize(14)


def test_variants_compiled_for_workload_lengths():
    for n in (256, 1000, 1024, 1536, 4096, 6000, 16384):
        assert fs.variant_count(n) >= 2, n


def test_two_pass_splits_are_balanced_and_tiled():
    """Every two-pass length gets the most balanced split whose column and
    row lengths have compiled tiles (radix-32 tiles included)."""
    for k in range(15, 23):
        n = 1 << k
        info = fs.split_info(n)
        assert info is not None, n
        n1, n2, nc, nr = info
        assert n1 * n2 == n and abs(n1.bit_length() - n2.bit_length()) <= 1, (n, n1, n2)
        assert n1 <= n2 and nc >= 1 and nr >= 1
    assert fs.split_info(1 << 20)[:2] == (1024, 1024)
    assert fs.split_info(1 << 16)[:2] == (256, 256)
    assert fs.split_info(1 << 17)[:2] == (256, 512)


def test_split_info_and_forced_variants_are_checked():
    assert fs.split_info(4096) is None            # single pass
    assert fs.split_info(3 ** 9) is None          # radix-stage fallback
    n1, n2, nc, nr = fs.split_info(1 << 20)
    assert n1 * n2 == 1 << 20 and nc >= 2 and nr >= 2
    with pytest.raises(fs.FFTError) as e:
        fs.Plan(4096, 4, split_variants=(0, 0))
    assert e.value.name == "FFT_ERR_INVALID_ARG"
    with pytest.raises(fs.FFTError):
        fs.Plan(1 << 20, 4, split_variants=(nc, 0))
    with pytest.raises(fs.FFTError):
        fs.Plan(4096, 4, variant=fs.variant_count(4096) + 3)


@pytest.mark.parametrize("args,status", [
    ((7, 4, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),      # odd
    ((2, 4, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),      # below the smallest real kernel
    ((2 * 7 * 64, 4, -1), "FFT_ERR_UNSUPPORTED_LENGTH"),
    ((1024, 0, -1), "FFT_ERR_INVALID_ARG"),
    ((1024, 4, 3), "FFT_ERR_INVALID_ARG"),
])
def test_real_create_rejects_bad_arguments(args, status):
    with pytest.raises(fs.FFTError) as ei:
        fs.RealPlan(*args)
    assert ei.value.name == status


def test_null_plan_frames_and_real():
    L = fs.lib()
    assert L.fft_exec_frames(None, None, 0, None, 1, 1, None, None) == -1
    assert fs.last_error()


def _work(entries):
    import numpy as np
    ent = np.zeros(len(entries), dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                                        ("segment_len", "<u4"), ("job", "<u4")])
    for i, (a, b, n) in enumerate(entries):
        ent[i] = (a, b, n, 0)
    return ent


@pytest.mark.parametrize("entries,ok", [
    # a job's run of segments, then another run
    ([(0, 0, 1024), (1024, 1024, 1024), (1024, 1024, 1024)], False),   # repeated output
    ([(0, 0, 1024), (1024, 1024, 1024), (4096, 4096, 4096)], True),
    ([(0, 0, 4096), (4096, 4096, 4096), (6000, 7000, 1024)], False),    # inside run 1's output
    ([(0, 8192, 4096), (4096, 12288, 4096), (0, 16384, 256)], True),    # inputs may overlap
    ([(0, 100, 256), (256, 356, 256), (512, 0, 256)], False),           # [0,256) vs [100,..)
])
def test_worklist_output_overlap_checked_on_runs(entries, ok):
    """Entries are grouped into runs for the range checks; overlaps between
    outputs of different runs, or inside what looks like a run, are found
    before any device work (a valid list then fails only for the missing
    device)."""
    with pytest.raises(fs.FFTError) as e:
        fs.WorkList(_work(entries))
    if ok:
        assert e.value.name in ("FFT_ERR_HIP", "FFT_ERR_OUT_OF_MEMORY"), e.value
    else:
        assert e.value.name == "FFT_ERR_OVERLAP", e.value


def test_one_call_worklist_checks_arguments():
    """The one-call form refuses a bad direction or a NULL list before it
    looks for a device."""
    L = fs.lib()
    assert L.fft_exec_worklist(None, 3, -1, None, None, None) == -1
    ent = _work([(0, 0, 1024)])
    items = ent.ctypes.data_as(ctypes.POINTER(fs.WorkItem))
    assert L.fft_exec_worklist(items, 1, 0, None, None, None) == -1
    assert "direction" in fs.last_error()
    assert L.fft_worklist_cache_clear() == 0
