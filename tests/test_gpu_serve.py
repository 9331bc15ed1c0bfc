"""Continuous-batching server on the GPU: every job's spectra are the same
alone and in the mix (bitwise, and within the bound), match the oracle,
and the mix really was packed into shared launches."""
import copy

import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs
from paper_1407_6915_amd.serve import GpuExecutor, JobState, serve
from siggen import workloads

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def make_jobs(n_jobs, seed_offset=7):
    import torch
    lengths = [1024, 4096, 65536, 1 << 20]
    rng = np.random.default_rng(seed_offset)
    jobs, keep = [], []
    for i in range(n_jobs):
        n = lengths[i % len(lengths)]
        n_seg = int(rng.integers(1, 4 if n == 1 << 20 else 12))
        wj = workloads.Job(i, 0.0002 * i, n, n_seg)
        x = workloads.job_signal(wj, seed_offset).segments(0, n_seg).reshape(-1)
        hin = torch.from_numpy(x).pin_memory()
        hout = torch.zeros_like(hin).pin_memory()
        keep += [hin, hout]
        jobs.append(JobState(i, wj.arrival_s, n, n_seg, hin.data_ptr(), hout.data_ptr()))
    return jobs, keep


def test_alone_equals_mix_and_matches_oracle():
    import torch
    announce("serving: mix vs alone")
    jobs, keep = make_jobs(24)
    arena = sum(j.samples for j in jobs) + 64 * len(jobs)
    ex = GpuExecutor(arena)
    st = serve(jobs, ex, arena)
    assert st["completed"] == len(jobs)
    assert len(ex.launches) < len(jobs), ex.launches        # the mix shared launches
    mix = {j.index: keep[2 * j.index + 1].numpy().copy() for j in jobs}
    bitwise = 0
    for j in jobs:
        solo = copy.copy(j)
        solo.arrival_s, solo.status, solo.tokens = 0.0, "pending", {}
        keep[2 * j.index + 1].zero_()
        ex_alone = GpuExecutor(j.samples + 64)
        s2 = serve([solo], ex_alone, j.samples + 64)
        assert s2["completed"] == 1 and len(ex_alone.launches) == 1
        alone = keep[2 * j.index + 1].numpy().reshape(j.n_seg, j.seg_len)
        m = mix[j.index].reshape(j.n_seg, j.seg_len)
        e = oracle.rel_l2(m, alone.astype(np.complex128))
        assert np.all(e <= oracle.tolerance(j.seg_len)), (j.index, e.max())
        bitwise += int(np.array_equal(m, alone))
        # one segment per job against the oracle
        x = keep[2 * j.index].numpy().reshape(j.n_seg, j.seg_len)
        s = j.n_seg - 1
        ref = oracle.fft_recursive(x[s], j.seg_len)
        assert oracle.rel_l2(m[s][None], ref)[0] <= oracle.tolerance(j.seg_len)
    print("  %d of %d jobs bitwise identical alone and in the mix" % (bitwise, len(jobs)),
          flush=True)
    assert bitwise == len(jobs)


def test_reserved_capacity_then_serving():
    announce("serving: reserved work-list capacity inside an HBM budget")
    jobs, keep = make_jobs(8, seed_offset=11)
    need = sum(j.samples for j in jobs) + 64 * len(jobs)
    budget = need * 8 + (1 << 30)
    ex = GpuExecutor(max_launch_samples=1 << 22, hbm_budget_bytes=budget)
    # the reserved work list (arrays, two-pass scratch, the 2^20-point
    # plan) counts against the budget; the arena gets the rest
    assert ex.resident_bytes > (1 << 22) * 8
    assert 0 <= budget - (ex.arena_samples * 8 + ex.resident_bytes) < 8
    arena = ex.arena_samples
    st = serve(jobs, ex, arena, max_launch_samples=1 << 22)
    assert st["completed"] + st["rejected"] == len(jobs)
    for j in jobs:
        if j.status != "done":
            continue
        x = keep[2 * j.index].numpy().reshape(j.n_seg, j.seg_len)
        y = keep[2 * j.index + 1].numpy().reshape(j.n_seg, j.seg_len)
        ref = oracle.fft_recursive(x[0], j.seg_len)
        assert oracle.rel_l2(y[0][None], ref)[0] <= oracle.tolerance(j.seg_len)


def test_budget_smaller_than_the_mix():
    announce("serving: tight budget")
    jobs, keep = make_jobs(12, seed_offset=9)
    biggest = max(j.samples for j in jobs)
    arena = biggest + 64                                      # one job at a time fits
    ex = GpuExecutor(arena)
    st = serve(jobs, ex, arena)
    assert st["completed"] == len(jobs) and st["peak_arena_samples"] <= arena
    for j in jobs:
        x = keep[2 * j.index].numpy().reshape(j.n_seg, j.seg_len)
        y = keep[2 * j.index + 1].numpy().reshape(j.n_seg, j.seg_len)
        ref = oracle.fft_recursive(x[0], j.seg_len)
        assert oracle.rel_l2(y[0][None], ref)[0] <= oracle.tolerance(j.seg_len)
