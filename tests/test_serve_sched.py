"""The serving scheduler on a virtual clock (no GPU): arena accounting,
admission by budget in arrival order, continuous batching, rejection of
jobs that can never fit, latency accounting."""
import math
import random

import numpy as np
import pytest

from paper_1407_6915_amd.serve import ALIGN, Arena, JobState, SimExecutor, serve
from siggen import workloads


def test_arena_first_fit_and_merge():
    a = Arena(1000 * ALIGN)
    offs = [a.alloc(100 * ALIGN) for _ in range(10)]
    assert offs == [i * 100 * ALIGN for i in range(10)]
    assert a.alloc(1) is None                       # full
    for o in offs[::2]:
        a.release(o, 100 * ALIGN)
    assert a.alloc(150 * ALIGN) is None             # fragmented: no 150 hole
    for o in offs[1::2]:
        a.release(o, 100 * ALIGN)
    assert a.free == [[0, 1000 * ALIGN]] and a.used == 0
    assert a.alloc(1000 * ALIGN) == 0


def test_arena_random_consistency():
    rng = random.Random(3)
    cap = 1 << 20
    a = Arena(cap)
    live = {}
    for _ in range(5000):
        if live and rng.random() < 0.5:
            o = rng.choice(list(live))
            a.release(o, live.pop(o))
        else:
            n = rng.randint(1, 50000)
            o = a.alloc(n)
            if o is not None:
                size = -(-n // ALIGN) * ALIGN
                for p, q in live.items():             # no overlap with live blocks
                    assert o + size <= p or p + -(-q // ALIGN) * ALIGN <= o
                assert o + size <= cap
                live[o] = n
        assert a.used == sum(-(-q // ALIGN) * ALIGN for q in live.values())
        assert a.used + sum(f[1] for f in a.free) == cap


def jobs_from(rate, n, cap=1 << 30):
    return [JobState(j.index, j.arrival_s, j.seg_len, j.n_seg)
            for j in workloads.serving_jobs(rate, n, cap_samples=cap)]


@pytest.mark.parametrize("rate", [5.0, 200.0, 2000.0])
def test_every_job_completes_within_budget(rate):
    jobs = jobs_from(rate, 400)
    ex = SimExecutor(link_gbs=50, hbm_gbs=5000)
    budget = 200 * 2 ** 30 // 8                      # 200 GiB of samples
    st = serve(jobs, ex, budget)
    assert st["completed"] == 400 and st["rejected"] == 0
    assert st["peak_arena_samples"] <= budget
    for j in jobs:
        assert j.admitted_s >= j.arrival_s - 1e-12
        assert j.done_s > j.admitted_s
        # no job can finish faster than its own two host-link copies
        assert j.done_s - j.arrival_s >= 2 * j.samples * 8 / 50e9 - 1e-9
    # admission in arrival order
    adm = [j.admitted_s for j in jobs]
    assert all(adm[i] <= adm[i + 1] + 1e-12 for i in range(len(adm) - 1))
    # every job is in exactly one launch
    seen = [k for launch in ex.launches for k in launch]
    assert sorted(seen) == list(range(400))


def test_continuous_batching_packs_under_load():
    light = jobs_from(2.0, 100)
    ex = SimExecutor()
    serve(light, ex, 1 << 40)
    assert len(ex.launches) == 100                  # idle GPU: one launch per job
    heavy = jobs_from(5000.0, 400)
    ex2 = SimExecutor()
    st = serve(heavy, ex2, 1 << 40)
    assert st["completed"] == 400
    assert len(ex2.launches) < 400                  # jobs that arrive meanwhile share launches
    assert max(len(l) for l in ex2.launches) > 1


def test_lone_job_is_dispatched_behind_its_copy():
    """At light load each job goes to the transform stream when it is
    admitted, ordered after its own copy on the device, so its latency is
    exactly copy in + transform + copy out."""
    jobs = jobs_from(1.0, 50)
    ex = SimExecutor(link_gbs=50, hbm_gbs=5000, launch_us=10)
    serve(jobs, ex, 1 << 40)
    assert len(ex.launches) == 50
    for j, launch, t_issue in zip(jobs, ex.launches, ex.issued):
        assert launch == [j.index]
        assert t_issue == pytest.approx(j.admitted_s)
        link = j.samples * 8 / 50e9
        passes = j.samples * (2 if j.seg_len > 16384 else 1)
        expect = 2 * link + 10e-6 + 16.0 * passes / 5000e9
        assert j.done_s - j.arrival_s == pytest.approx(expect, rel=1e-9, abs=1e-12)


def test_small_budget_serialises_but_completes():
    jobs = [JobState(i, 0.001 * i, 4096, 256) for i in range(40)]   # 1M samples each
    ex = SimExecutor()
    budget = 3 * 4096 * 256                              # room for three jobs
    st = serve(jobs, ex, budget)
    assert st["completed"] == 40
    assert st["peak_arena_samples"] <= budget


def test_oversized_job_is_rejected_not_stuck():
    jobs = [JobState(0, 0.0, 4096, 16), JobState(1, 0.0, 1 << 20, 64),
            JobState(2, 0.001, 4096, 16)]
    ex = SimExecutor()
    st = serve(jobs, ex, (1 << 20) * 8)             # job 1 (64 M samples) never fits
    assert st["rejected"] == 1 and jobs[1].status == "rejected"
    assert jobs[0].status == "done" and jobs[2].status == "done"
