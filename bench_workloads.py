"""The other workloads of bench.py (``--workload small|uneven|streamed|
serving|long|real|frames``).  Each prints one JSON line.  All inputs are seeded synthetic
signals (siggen); device buffers come from torch; every transform runs in
libfftseg's kernels."""
from __future__ import annotations

import ctypes
import json
import math
import time

import numpy as np

FLOP = lambda n: 5.0 * n * math.log2(n) if n > 1 else 0.0  # noqa: E731


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(torch, fn, reps, warmup=2):
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def small(args):
    import torch
    import paper_1407_6915_amd as fs
    from siggen import workloads
    n, b = workloads.SMALL["seg_len"], workloads.SMALL["batch"]
    x = workloads.small_signal().segments(0, b)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    yd = torch.empty_like(xd)
    sh = torch.cuda.current_stream().cuda_stream
    with fs.Plan(n, b) as p:
        t = _time(torch, lambda: p.exec_ptr(xd.data_ptr(), yd.data_ptr(), sh), args.steps)
        tg = _time(torch, lambda: p.exec_graph_ptr(xd.data_ptr(), yd.data_ptr(), sh), args.steps)
    # where a graph pays: launch sequences, small enough that launching
    # them costs more than running them: a two-pass plan of 16 segments of
    # 65536 points split into 2-segment sub-batches (16 launches), and a
    # small mixed work list (8 segments of each length: one launch per
    # one-pass length, the wide tiles, the two work-list launches)
    import os
    seqs = {}
    m = 1 << 16
    xm = torch.randn(16 * m, dtype=torch.complex64, device="cuda")
    ym = torch.empty_like(xm)
    os.environ["FFTSEG_SUB_SAMPLES"] = str(2 * m)
    try:
        with fs.Plan(m, 16) as p:
            te = _time(torch, lambda: p.exec_ptr(xm.data_ptr(), ym.data_ptr(), sh), args.steps)
            tgr = _time(torch, lambda: p.exec_graph_ptr(xm.data_ptr(), ym.data_ptr(), sh),
                        args.steps)
    finally:
        del os.environ["FFTSEG_SUB_SAMPLES"]
    seqs["plan_65536x16_in_8_sub_batches"] = {"launches": 16, "us_per_exec": round(te * 1e6, 2),
                                              "us_per_graph_exec": round(tgr * 1e6, 2)}
    lens = np.repeat(np.asarray(workloads.UNEVEN_LENGTHS, np.int64), 8)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    ent = np.zeros(len(lens), dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                                     ("segment_len", "<u4"), ("job", "<u4")])
    ent["in_off"] = ent["out_off"] = offs
    ent["segment_len"] = lens
    xw = torch.randn(int(lens.sum()), dtype=torch.complex64, device="cuda")
    yw = torch.empty_like(xw)
    with fs.WorkList(ent) as wl:
        te = _time(torch, lambda: wl.exec_ptr(xw.data_ptr(), yw.data_ptr(), sh), args.steps)
        tgr = _time(torch, lambda: wl.exec_ptr(xw.data_ptr(), yw.data_ptr(), sh, graph=True),
                    args.steps)
    seqs["worklist_8_segments_per_length"] = {"us_per_exec": round(te * 1e6, 2),
                                              "us_per_graph_exec": round(tgr * 1e6, 2)}
    print(json.dumps({"workload": workloads.SMALL["name"], "segment_len": n, "batch": b,
                      "us_per_exec": round(t * 1e6, 2), "us_per_graph_exec": round(tg * 1e6, 2),
                      "GFLOP/s": round(FLOP(n) * b / t / 1e9, 1),
                      "GB/s": round(16 * n * b / t / 1e9, 1),
                      "launch_sequences": seqs}), flush=True)
    return 0


def uneven(args):
    import torch
    import paper_1407_6915_amd as fs
    from siggen import workloads
    lengths = workloads.uneven_lengths()
    in_off = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    total = int(lengths.sum())
    sig = workloads.uneven_signal()
    xd = torch.empty(total, dtype=torch.complex64, device="cuda")
    chunk = 1 << 27
    for a in range(0, total, chunk):
        m = min(chunk, total - a)
        xd[a:a + m].copy_(torch.from_numpy(sig.samples(a, m)))
    yd = torch.empty_like(xd)
    ent = np.zeros(len(lengths), dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                                        ("segment_len", "<u4"), ("job", "<u4")])
    ent["in_off"] = ent["out_off"] = in_off
    ent["segment_len"] = lengths
    sh = torch.cuda.current_stream().cuda_stream
    fs.tune_clear()
    t_build = time.perf_counter()
    wl = fs.WorkList(ent)
    t_build = time.perf_counter() - t_build
    t_wl = _time(torch, lambda: wl.exec_ptr(xd.data_ptr(), yd.data_ptr(), sh), args.steps)
    t_graph = _time(torch, lambda: wl.exec_ptr(xd.data_ptr(), yd.data_ptr(), sh, graph=True),
                    args.steps)
    wl.status()
    desc = wl.describe()
    wl.close()
    # tuned: each one-pass length's plan variant, grid and work-list route
    # picked by fft_autotune on as many segments as the list holds of it
    t0 = time.perf_counter()
    tuned = {}
    for n in workloads.UNEVEN_LENGTHS:
        if args.no_tune or fs.indexed_count(n) == 0:
            continue
        c = int((lengths == n).sum())
        best = fs.autotune(n, c)
        tuned[str(n)] = best
    t_tune = time.perf_counter() - t0
    wl = fs.WorkList(ent)
    t_wl_t = _time(torch, lambda: wl.exec_ptr(xd.data_ptr(), yd.data_ptr(), sh), args.steps)
    t_graph_t = _time(torch, lambda: wl.exec_ptr(xd.data_ptr(), yd.data_ptr(), sh, graph=True),
                      args.steps)
    wl.status()
    desc_t = wl.describe()
    wl.close()
    fs.tune_clear()
    # reference from the packed layout: per length, gather its segments into
    # a contiguous batch, one plain launch, scatter the spectra back (every
    # length here is a multiple of 8 samples, so the gather moves 64-byte
    # rows)
    rows8 = {}
    for n in workloads.UNEVEN_LENGTHS:
        sel = torch.from_numpy(in_off[lengths == n].astype(np.int64) // 8).cuda()
        rows8[n] = (sel[:, None] + torch.arange(n // 8, device="cuda")[None, :]).reshape(-1)
    gplans = {n: fs.Plan(n, int((lengths == n).sum())) for n in workloads.UNEVEN_LENGTHS}
    xv, yv = xd.view(-1, 8), yd.view(-1, 8)

    def gather_plain_scatter():
        for n, idx in rows8.items():
            xs = xv.index_select(0, idx)
            ys = torch.empty_like(xs)
            gplans[n].exec_ptr(xs.data_ptr(), ys.data_ptr(), sh)
            yv.index_copy_(0, idx, ys)
    t_gps = _time(torch, gather_plain_scatter, max(3, args.steps // 3))
    for p in gplans.values():
        p.close()
    del rows8, xv, yv
    # reference: one plain batched launch per length over length-sorted data
    per_len = {}
    bufs = {}
    for n in workloads.UNEVEN_LENGTHS:
        c = int((lengths == n).sum())
        xs = torch.randn(c * n, dtype=torch.complex64, device="cuda")
        bufs[n] = (xs, torch.empty_like(xs), fs.Plan(n, c))
    del xd, yd

    def all_lengths():
        for n, (xs, ys, p) in bufs.items():
            p.exec_ptr(xs.data_ptr(), ys.data_ptr(), sh)
    t_plain = _time(torch, all_lengths, args.steps)
    for n, (xs, ys, p) in bufs.items():
        per_len[str(n)] = round(_time(torch, lambda: p.exec_ptr(xs.data_ptr(), ys.data_ptr(), sh),
                                      max(3, args.steps // 4)) * 1e3, 3)
        p.close()
    flops = float(sum(FLOP(int(n)) for n in lengths))
    comp = 16.0 * total
    plan_bytes = float(sum(16 * n * (2 if n == 65536 else 1) for n in lengths))
    out = {"workload": workloads.UNEVEN["name"], "segments": len(lengths), "samples": total,
           "worklist": desc, "build_s": round(t_build, 3),
           "persistent_ms": round(t_wl * 1e3, 3), "persistent_graph_ms": round(t_graph * 1e3, 3),
           "tuned": {"persistent_ms": round(t_wl_t * 1e3, 3),
                     "persistent_graph_ms": round(t_graph_t * 1e3, 3),
                     "indexed": desc_t.get("indexed"), "tune_s": round(t_tune, 1),
                     "best_us_per_length": tuned},
           "per_length_plain_ms": round(t_plain * 1e3, 3), "per_length_ms": per_len,
           "per_length_from_packed_ms": round(t_gps * 1e3, 3),
           "per_length_from_packed_note": "gather each length's segments (index_select of "
                                         "64-byte rows), one plain launch, scatter back",
           "GFLOP/s": {"persistent": round(flops / t_wl / 1e9, 1),
                       "persistent_graph": round(flops / t_graph / 1e9, 1),
                       "per_length_plain": round(flops / t_plain / 1e9, 1)},
           "compulsory_GB/s": {"persistent": round(comp / t_wl / 1e9, 1),
                               "per_length_plain": round(comp / t_plain / 1e9, 1)},
           "plan_GB/s_persistent": round(plan_bytes / t_wl / 1e9, 1),
           "roofline_frac_compulsory": round(comp / t_wl / 1e9 / 8000.0, 4)}
    print(json.dumps(out), flush=True)
    return 0


def streamed(args):
    """The 2^20-point workload streamed from the host: chunks of 512 segments
    (4 GiB), ``args.chunks`` of them (64 = 32768 segments, 256 GiB).

    No torch allocation is made here: the plan, its pinned slots and device
    ring, and the pinned pool all belong to the library and are released
    before this returns, so nothing HIP-related is left for process exit.

    (1) link reference: a pool of 4 pre-generated pinned chunks cycled
        through the pipeline (no host work per chunk);
    (2) as configured: every chunk generated from the seed by the fill
        callback; the drain callback sums every output segment's energy and
        keeps the first and last segment of each chunk.
    Checks: Parseval on every segment, and the oracle on the two kept
    segments of every chunk (timed: the CPU baseline of this workload).
    """
    import oracle
    import paper_1407_6915_amd as fs
    from siggen import workloads
    n, seg = workloads.LONG["seg_len"], workloads.LONG["chunk_segments"]
    chunks = args.chunks
    chunk_samples = n * seg
    nbytes = chunk_samples * 8
    tol = 5e-7 * math.log2(n)                  # per-segment rel-L2 bound
    parseval_bound = 2.0 * tol + tol * tol     # |E_out / (N E_in) - 1| it implies
    sig = workloads.long_signal()
    plan = fs.Plan(n, seg)

    # (1) link reference over a pool of pre-generated pinned chunks
    pool = min(4, chunks)
    t0 = time.perf_counter()
    ins = [fs.HostBuffer(nbytes) for _ in range(pool)]
    outs = [fs.HostBuffer(nbytes) for _ in range(pool)]
    for c in range(pool):
        sig.fill_ptr(c * chunk_samples, chunk_samples, ins[c].ptr)
    t_pool = time.perf_counter() - t0
    st = plan.exec_stream_pinned(chunks, [b.ptr for b in ins], [b.ptr for b in outs], 3)
    tl_pool = plan.stream_timeline()
    # Parseval on the pool's last round of outputs
    from siggen import segment_energy
    pool_dev = 0.0
    for c in range(max(0, chunks - pool), chunks):
        slot = c % pool
        e_in = segment_energy(ins[slot].view().reshape(seg, n))
        e_out = segment_energy(outs[slot].view().reshape(seg, n))
        pool_dev = max(pool_dev, float(np.max(np.abs(e_out / (n * e_in) - 1.0))))
    for b in ins + outs:
        b.close()

    # (2) as configured: generated from the seed, every segment checked
    # fill and drain each use every host thread (they run at once, on
    # different threads of this process): giving the drain a fixed share
    # of the threads slowed the compute-bound fill by more than the
    # overlap gained (11.6-11.8 s against 9.2 s for the 64 chunks)
    fill, drain, src, chk = sig.checked_chunk_source(seg, chunks)
    rc, failed, stg = plan.exec_stream(chunks, (fill, src), (drain, src), 3)
    tl_gen = plan.stream_timeline()
    plan.close()
    if rc != 0:
        raise RuntimeError("streamed run failed at chunk %s (status %d)" % (failed, rc))
    dev = np.abs(chk.energy_out / (n * chk.energy_in) - 1.0)

    # CPU baseline: the oracle on the first and last segment of every chunk,
    # inputs regenerated from the seed
    idx = [c * seg + s for c in range(chunks) for s in (0, seg - 1)]
    xs = np.concatenate([sig.segments(i, 1) for i in idx])
    t0 = time.perf_counter()
    ref = oracle.fft_recursive(xs, n)
    t_oracle = time.perf_counter() - t0
    errs = oracle.rel_l2(chk.saved_out.reshape(-1, n), ref)
    del xs, ref

    import bench_profile
    overlap = {}
    md = ["# Streamed 2^20-point chunks: copy/compute overlap", "",
          "Command (run from the repository root):", "",
          "    python3 bench.py --workload streamed --chunks %d --overlap-md %s"
          % (chunks, args.overlap_md), "",
          "Chunks of 512 segments (4 GiB each way).  Intervals from the pipeline's HIP events "
          "on its three streams (copy in, transform, copy out), read back on the GPU clock "
          "with fft_stream_last_timeline, in ms from chunk 0's copy-in start.", ""]
    for key, title, tl in (("link_reference", "Pool of pre-generated pinned chunks "
                            "(link reference)", tl_pool),
                           ("as_configured", "Every chunk generated from the seed "
                            "(as configured)", tl_gen)):
        H, K, D = bench_profile.timeline_intervals(tl)
        overlap[key] = {k: round(v, 4) for k, v in
                        bench_profile.overlap_stats(H, [iv for ks in K for iv in ks], D).items()}
        md += bench_profile.overlap_lines(title, H, K, D, nbytes)
    if args.overlap_md:
        open(args.overlap_md, "w").write("\n".join(md) + "\n")

    link_wall = st["wall_s"]
    gen_wall = stg["wall_s"]
    host_s = stg["fill_s"] + stg["drain_s"]
    out = {"workload": workloads.LONG["name"], "segment_len": n, "segments_per_chunk": seg,
           "chunk_bytes": nbytes, "chunks": chunks, "segments": chunks * seg,
           "signal_bytes": chunks * nbytes,
           "as_configured": {
               "input": "every chunk generated on the host from the seed, in the fill "
                        "callback, into the library's pinned slots",
               "wall_s": round(gen_wall, 3),
               "host_link_GBps_each_way": round(stg["bytes_h2d"] / gen_wall / 1e9, 2),
               "GFLOP/s": round(FLOP(n) * seg * chunks / gen_wall / 1e9, 1),
               "fill_s": round(stg["fill_s"], 3),
               "generation_GBps": round(stg["bytes_h2d"] / max(stg["fill_s"], 1e-9) / 1e9, 2),
               "drain_s": round(stg["drain_s"], 3),
               "drain_note": "per-segment output energies (Parseval) and the kept segments, "
                             "on a worker thread, overlapping the fill",
               "h2d_s": round(stg["h2d_s"], 3), "d2h_s": round(stg["d2h_s"], 3),
               "transform_s": round(stg["compute_s"], 3),
               "bound_by": ("host generation and checks" if host_s > 0.8 * gen_wall and
                            gen_wall > 1.2 * link_wall else "host link"),
               "overlap": overlap["as_configured"]},
           "link_reference": {
               "input": "%d pre-generated pinned chunks cycled" % pool,
               "wall_s": round(link_wall, 3),
               "host_link_GBps_each_way": round(st["bytes_h2d"] / link_wall / 1e9, 2),
               "host_link_GBps_total": round(2.0 * st["bytes_h2d"] / link_wall / 1e9, 2),
               "h2d_GBps_per_copy": round(st["bytes_h2d"] / max(st["h2d_s"], 1e-9) / 1e9, 2),
               "d2h_GBps_per_copy": round(st["bytes_d2h"] / max(st["d2h_s"], 1e-9) / 1e9, 2),
               "h2d_s": round(st["h2d_s"], 3), "d2h_s": round(st["d2h_s"], 3),
               "transform_s": round(st["compute_s"], 3),
               "transform_HBM_GBps": round(32.0 * chunk_samples * chunks /
                                           max(st["compute_s"], 1e-9) / 1e9, 1),
               "GFLOP/s": round(FLOP(n) * seg * chunks / link_wall / 1e9, 1),
               "amdahl_parallel_fraction": round(st["compute_s"] /
                                                 (st["compute_s"] + st["h2d_s"]), 4),
               "pool_fill_s": round(t_pool, 2),
               "parseval_max_rel_dev_last_round": pool_dev,
               "overlap": overlap["link_reference"]},
           "checks": {
               "parseval_segments": int(dev.size),
               "parseval_max_rel_dev": float(dev.max()),
               "parseval_bound": parseval_bound,
               "parseval_over_bound": int((dev > parseval_bound).sum()),
               "oracle_segments": len(idx),
               "oracle_max_rel_l2": float(errs.max()),
               "oracle_mean_rel_l2": float(errs.mean()),
               "rel_l2_bound": tol,
               "oracle_over_bound": int((errs > tol).sum())},
           "cpu_baseline": {
               "value": round(FLOP(n) * len(idx) / t_oracle / 1e9, 3), "unit": "GFLOP/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": "first and last segment of each of the %d chunks (%d x 2^20 "
                         "points, %.1f s, FP64 recursive radix-2/3/5 DFT)"
                         % (chunks, len(idx), t_oracle)}}
    print(json.dumps(out), flush=True)
    ok = out["checks"]["parseval_over_bound"] == 0 and out["checks"]["oracle_over_bound"] == 0
    return 0 if ok else 1


def serving(args):
    import torch
    import paper_1407_6915_amd as fs
    from paper_1407_6915_amd.serve import GpuExecutor, JobState, serve, serve_fifo
    from siggen import workloads
    rng = np.random.default_rng(5)
    pool_samples = 1 << 32                                 # 32 GiB pinned payload pool
    t0 = time.perf_counter()
    pool = torch.empty(pool_samples, dtype=torch.complex64, pin_memory=True)
    outp = torch.empty(pool_samples, dtype=torch.complex64, pin_memory=True)
    gen = workloads.job_signal(workloads.Job(0, 0.0, 4096, 1))
    chunk = 1 << 28
    for a in range(0, pool_samples, chunk):
        gen.fill_ptr(a, chunk, pool.data_ptr() + a * 8)
    t_pool = time.perf_counter() - t0
    base_in, base_out = pool.data_ptr(), outp.data_ptr()

    def job_states(rate, n_jobs, off):
        js = []
        for j in workloads.serving_jobs(rate, n_jobs, seed_offset=off):
            start = int(rng.integers(0, pool_samples - j.samples)) & ~63
            js.append(JobState(j.index, j.arrival_s, j.seg_len, j.n_seg,
                               base_in + start * 8, base_out + start * 8))
        return js

    lengths = workloads.SERVING_LENGTHS
    cap = 1 << 30
    plans = {n: fs.Plan(n, cap // n) for n in lengths}
    fifo_arena = torch.empty(cap, dtype=torch.complex64, device="cuda")
    budget_bytes = 200 * 10 ** 9
    max_launch = 1 << 31                                   # bounds the two-pass scratch
    # the arena gets what the work list's reserved device memory leaves
    ex = GpuExecutor(max_launch_samples=max_launch, hbm_budget_bytes=budget_bytes)
    arena_samples = ex.arena_samples
    # saturation: the same jobs, every one queued at t = 0, through each path
    sat_f = job_states(1e9, min(args.jobs, 300), 99)
    sat_c = [JobState(j.index, j.arrival_s, j.seg_len, j.n_seg, j.host_in, j.host_out)
             for j in sat_f]
    st_sat = serve_fifo(sat_f, plans, fifo_arena)
    lam_sat = st_sat["jobs_per_s"]
    ex.t0 = time.perf_counter()
    st_sat_c = serve(sat_c, ex, arena_samples, max_launch_samples=max_launch,
                     max_copies_in_flight=args.inflight)
    rows = []
    for k, frac in enumerate(float(r) for r in args.rates.split(",")):
        lam = frac * lam_sat
        jobs_c = job_states(lam, args.jobs, 10 + k)
        jobs_f = [JobState(j.index, j.arrival_s, j.seg_len, j.n_seg, j.host_in, j.host_out)
                  for j in jobs_c]
        ex.t0 = time.perf_counter()
        ex.launches.clear()
        sc = serve(jobs_c, ex, arena_samples, max_launch_samples=max_launch,
                   max_copies_in_flight=args.inflight)
        sf = serve_fifo(jobs_f, plans, fifo_arena)
        rows.append({"rate_frac": frac, "rate_jobs_per_s": round(lam, 2),
                     "continuous": {key: round(sc[key], 3) for key in
                                    ("jobs_per_s", "p50_ms", "p99_ms", "mean_ms")} |
                     {"launches": sc["launches"], "GB/s_payload":
                      round(sc["samples_per_s"] * 8 / 1e9, 2)},
                     "plain_fifo": {key: round(sf[key], 3) for key in
                                    ("jobs_per_s", "p50_ms", "p99_ms", "mean_ms")}})
        print(json.dumps({"progress": rows[-1]}), flush=True)
    for p in plans.values():
        p.close()
    print(json.dumps({"workload": "serving", "jobs_per_rate": args.jobs,
                      "copies_in_flight": args.inflight,
                      "plain_saturation_jobs_per_s": round(lam_sat, 2),
                      "continuous_saturation_jobs_per_s": round(st_sat_c["jobs_per_s"], 2),
                      "saturation_payload_GBps": {
                          "plain": round(st_sat["samples_per_s"] * 8 / 1e9, 2),
                          "continuous": round(st_sat_c["samples_per_s"] * 8 / 1e9, 2)},
                      "hbm_budget_bytes": budget_bytes,
                      "device_footprint_bytes": arena_samples * 8 + ex.resident_bytes,
                      "worklist_resident_bytes": ex.resident_bytes,
                      "pool_fill_s": round(t_pool, 2),
                      "rates": rows}), flush=True)
    return 0


def long(args):
    """Four-step transforms resident in HBM: 8 GiB batches of 65536- and
    2^20-point segments (the kernel side of the streamed workload)."""
    import torch
    import paper_1407_6915_amd as fs
    total = 1 << 30
    g = torch.Generator(device="cuda").manual_seed(0x14076915)
    x = torch.randn(total, dtype=torch.complex64, device="cuda", generator=g)
    y = torch.empty_like(x)
    sh = torch.cuda.current_stream().cuda_stream
    rows = []
    for n in (1 << 16, 1 << 20):
        b = total // n
        with fs.Plan(n, b) as p:
            t = _time(torch, lambda: p.exec_ptr(x.data_ptr(), y.data_ptr(), sh), args.steps)
            d = p.describe()
        rows.append({"segment_len": n, "batch": b, "ms": round(t * 1e3, 3),
                     "GFLOP/s": round(FLOP(n) * b / t / 1e9, 1),
                     "algorithmic_GBps": round(16.0 * total / t / 1e9, 1),
                     "two_pass_traffic_GBps": round(32.0 * total / t / 1e9, 1),
                     "split": [d["n1"], d["n2"]],
                     "tile_variants": [d["column_variant"], d["row_variant"]],
                     "grid_mult": d["grid_mult"]})
    print(json.dumps({"workload": "long_in_hbm", "rows": rows}), flush=True)
    return 0


def real(args):
    """Real float32 segments (the 4-byte samples of the paper's records):
    1024-point segments over 2^30 real samples (4 GiB in), forward to bins
    0..512 and back, next to the complex transform of the same samples
    stored as complex64 with zero imaginary parts."""
    import torch
    import paper_1407_6915_amd as fs
    n, total = 1024, 1 << 30
    b = total // n
    g = torch.Generator(device="cuda").manual_seed(0x14076916)
    x = torch.randn(total, dtype=torch.float32, device="cuda", generator=g)
    spec = torch.empty(b * (n // 2 + 1), dtype=torch.complex64, device="cuda")
    back = torch.empty_like(x)
    sh = torch.cuda.current_stream().cuda_stream
    fwd_bytes = b * (n * 4 + (n // 2 + 1) * 8)
    with fs.RealPlan(n, b, fs.FORWARD) as pf, fs.RealPlan(n, b, fs.INVERSE) as pi:
        tf = _time(torch, lambda: pf.exec_ptr(x.data_ptr(), spec.data_ptr(), sh), args.steps)
        ti = _time(torch, lambda: pi.exec_ptr(spec.data_ptr(), back.data_ptr(), sh), args.steps)
    del back
    xc = x.to(torch.complex64)
    yc = torch.empty_like(xc)
    with fs.Plan(n, b) as pc:
        tc = _time(torch, lambda: pc.exec_ptr(xc.data_ptr(), yc.data_ptr(), sh), args.steps)
    # 2^21-point segments of the same samples: the 2^20-point half runs as a
    # two-pass plan and the even/odd split as a separate pass
    nl = 1 << 21
    bl = total // nl
    spec_l = torch.empty(bl * (nl // 2 + 1), dtype=torch.complex64, device="cuda")
    back_l = torch.empty_like(x)
    with fs.RealPlan(nl, bl, fs.FORWARD) as pf, fs.RealPlan(nl, bl, fs.INVERSE) as pi:
        tfl = _time(torch, lambda: pf.exec_ptr(x.data_ptr(), spec_l.data_ptr(), sh), args.steps)
        til = _time(torch, lambda: pi.exec_ptr(spec_l.data_ptr(), back_l.data_ptr(), sh),
                    args.steps)
    del back_l, spec_l
    with fs.Plan(nl, bl) as pc:
        tcl = _time(torch, lambda: pc.exec_ptr(xc.data_ptr(), yc.data_ptr(), sh), args.steps)
    long_row = {"segment_len": nl, "batch": bl, "forward_ms": round(tfl * 1e3, 3),
                "inverse_ms": round(til * 1e3, 3),
                "complex_same_samples_ms": round(tcl * 1e3, 3),
                "speedup_vs_complex": round(tcl / tfl, 2)}
    print(json.dumps({"workload": "real_n1024_b1048576", "segment_len": n, "batch": b,
                      "forward_ms": round(tf * 1e3, 3), "inverse_ms": round(ti * 1e3, 3),
                      "forward_GBps": round(fwd_bytes / tf / 1e9, 1),
                      "inverse_GBps": round(fwd_bytes / ti / 1e9, 1),
                      "bytes_per_real_sample": round(fwd_bytes / total, 3),
                      "complex_same_samples_ms": round(tc * 1e3, 3),
                      "speedup_vs_complex": round(tc / tf, 2),
                      "separate_split_n2097152": long_row}), flush=True)
    return 0


def frames(args):
    """Short-time transform: 4096-point frames every 1024 samples (75 %
    overlap) of a 2^28-sample signal with a periodic Hann window, next to
    the plain transform of as many disjoint segments."""
    import torch
    import paper_1407_6915_amd as fs
    n, hop, total = 4096, 1024, 1 << 28
    nf = (total - n) // hop + 1
    g = torch.Generator(device="cuda").manual_seed(0x14076917)
    x = torch.randn(total, dtype=torch.complex64, device="cuda", generator=g)
    j = torch.arange(n, dtype=torch.float64, device="cuda")
    w = (0.5 - 0.5 * torch.cos(2 * math.pi * j / n)).float()
    y = torch.empty(nf * n, dtype=torch.complex64, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    with fs.Plan(n, nf) as p:
        t = _time(torch, lambda: p.exec_frames_ptr(x.data_ptr(), total, y.data_ptr(), nf, hop,
                                                   w.data_ptr(), sh), args.steps)
        seg = total // n
        t_plain = _time(torch, lambda: p.exec_ptr(x.data_ptr(), y.data_ptr(), sh, seg),
                        args.steps)
    out_bytes = nf * n * 8
    # 65536-point frames every 16384 samples: read by the two-pass plan's
    # column pass (75 % overlap, Hann), next to as many disjoint segments
    n2, hop2 = 1 << 16, 1 << 14
    nf2 = (total - n2) // hop2 + 1
    j2 = torch.arange(n2, dtype=torch.float64, device="cuda")
    w2 = (0.5 - 0.5 * torch.cos(2 * math.pi * j2 / n2)).float()
    y2 = torch.empty(nf2 * n2, dtype=torch.complex64, device="cuda")
    with fs.Plan(n2, nf2) as p:
        t2 = _time(torch, lambda: p.exec_frames_ptr(x.data_ptr(), total, y2.data_ptr(), nf2,
                                                    hop2, w2.data_ptr(), sh), args.steps)
        seg2 = total // n2
        t2p = _time(torch, lambda: p.exec_ptr(x.data_ptr(), y2.data_ptr(), sh, seg2),
                    args.steps)
    del y2
    two_pass = {"segment_len": n2, "hop": hop2, "frames": nf2, "ms": round(t2 * 1e3, 3),
                "frame_bytes_two_pass_GBps": round(32.0 * nf2 * n2 / t2 / 1e9, 1),
                "plain_segments_ms": round(t2p * 1e3, 3),
                "plain_two_pass_GBps": round(32.0 * seg2 * n2 / t2p / 1e9, 1)}
    print(json.dumps({"workload": "frames_n4096_hop1024_hann", "segment_len": n, "hop": hop,
                      "frames": nf, "signal_samples": total, "ms": round(t * 1e3, 3),
                      "GFLOP/s": round(FLOP(n) * nf / t / 1e9, 1),
                      "frame_bytes_GBps": round(2 * out_bytes / t / 1e9, 1),
                      "min_hbm_bytes_GBps": round((total * 8 + out_bytes) / t / 1e9, 1),
                      "plain_segments_ms": round(t_plain * 1e3, 3),
                      "plain_GBps": round(16.0 * seg * n / t_plain / 1e9, 1),
                      "two_pass_n65536_hop16384": two_pass}), flush=True)
    return 0


def frame_lengths(args):
    """Frames of each listed length every N/4 samples (75 % overlap) of a
    2^28-sample signal with a periodic Hann window: the frame kernel of every
    one-pass length, or the column pass of two-pass lengths."""
    import torch
    import paper_1407_6915_amd as fs
    total = 1 << 28
    g = torch.Generator(device="cuda").manual_seed(0x14076917)
    x = torch.randn(total, dtype=torch.complex64, device="cuda", generator=g)
    sh = torch.cuda.current_stream().cuda_stream
    rows = []
    for n in [int(v) for v in args.lengths.split(",")]:
        hop = max(1, n // 4)
        nf = (total - n) // hop + 1
        j = torch.arange(n, dtype=torch.float64, device="cuda")
        w = (0.5 - 0.5 * torch.cos(2 * math.pi * j / n)).float()
        y = torch.empty(nf * n, dtype=torch.complex64, device="cuda")
        with fs.Plan(n, nf) as p:
            t = _time(torch, lambda: p.exec_frames_ptr(x.data_ptr(), total, y.data_ptr(), nf,
                                                       hop, w.data_ptr(), sh), args.steps)
            kind = p.describe()["kind"]
        rows.append({"segment_len": n, "hop": hop, "frames": nf, "kind": kind,
                     "ms": round(t * 1e3, 3), "GFLOP/s": round(FLOP(n) * nf / t / 1e9, 1),
                     "frame_bytes_GBps": round(16.0 * nf * n / t / 1e9, 1)})
        del y
    print(json.dumps({"workload": "frame_lengths_hop_quarter_hann", "signal_samples": total,
                      "rows": rows}), flush=True)
    return 0


def lengths(args):
    """Plain batched plans of the listed lengths, each over 8 GiB resident in
    HBM (the kernel-level rates behind the one-pass and two-pass rows; a
    driver for counter runs)."""
    import torch
    import paper_1407_6915_amd as fs
    total = 1 << 30
    g = torch.Generator(device="cuda").manual_seed(0x14076917)
    x = torch.randn(total, dtype=torch.complex64, device="cuda", generator=g)
    y = torch.empty_like(x)
    sh = torch.cuda.current_stream().cuda_stream
    rows = []
    for n in [int(v) for v in args.lengths.split(",") if v]:
        b = total // n
        with fs.Plan(n, b) as p:
            t = _time(torch, lambda: p.exec_ptr(x.data_ptr(), y.data_ptr(), sh), args.steps)
            d = p.describe()
        passes = 2 if d.get("kind") == "four_step" else 1
        rows.append({"segment_len": n, "batch": b, "kind": d.get("kind"),
                     "variant": d.get("variant"), "ms": round(t * 1e3, 3),
                     "GFLOP/s": round(FLOP(n) * b / t / 1e9, 1),
                     "algorithmic_GBps": round(16.0 * b * n / t / 1e9, 1),
                     "plan_traffic_GBps": round(16.0 * passes * b * n / t / 1e9, 1)})
    print(json.dumps({"workload": "lengths_in_hbm", "rows": rows}), flush=True)
    return 0


def _fs_type(path):
    """Filesystem type of the mount holding path (from /proc/mounts)."""
    import os
    path = os.path.realpath(path)
    best, kind = "", "unknown"
    try:
        for line in open("/proc/mounts"):
            parts = line.split()
            if len(parts) >= 3 and path.startswith(parts[1]) and len(parts[1]) > len(best):
                best, kind = parts[1], parts[2]
    except OSError:
        pass
    return kind


def file(args):
    """File in, file out (the paper's setting, Sec. III-IV): a signal file of
    4096-point segments on the box's local disk, read in 1 GiB chunks into
    the pinned ring, transformed, and each chunk's spectra written at the
    same offset of an output file.  The input is written first, flushed and
    dropped from the page cache, so the reads come from the device under the
    file system.  Reports read and write GB/s, host-link GB/s, transform
    time and the time shares, next to the paper's (FFT 5-8 % of the GPU
    run, I/O the rest)."""
    import os
    import shutil
    import paper_1407_6915_amd as fs
    from siggen import segment_energy, workloads
    n = workloads.LARGE["seg_len"]
    seg = 1 << 17                       # 1 GiB chunks
    chunk = n * seg * 8
    d = args.file_dir or os.environ.get("TMPDIR", "/tmp")
    free = shutil.disk_usage(d).free
    want = args.file_gib << 30
    size = min(want, max(0, (free - (8 << 30)) // 2) // chunk * chunk)
    if size < 2 * chunk:
        print(json.dumps({"workload": "file", "skipped": "only %.1f GiB free in %s"
                          % (free / 2 ** 30, d)}), flush=True)
        return 0
    chunks = size // chunk
    fin = os.path.join(d, "fftseg_bench_in_%d.bin" % os.getpid())
    fout = os.path.join(d, "fftseg_bench_out_%d.bin" % os.getpid())
    sig = workloads.large_signal()
    buf = fs.HostBuffer(chunk)
    try:
        t0 = time.perf_counter()
        fd = os.open(fin, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o644)
        try:
            v = buf.view()
            for c in range(chunks):
                sig.fill_ptr(c * n * seg, n * seg, buf.ptr)
                mv = memoryview(v.view(np.uint8))
                off = 0
                while off < chunk:
                    off += os.pwrite(fd, mv[off:], c * chunk + off)
            os.fsync(fd)
            os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)
        finally:
            os.close(fd)
        t_write_in = time.perf_counter() - t0
        with fs.Plan(n, seg) as plan:
            rc, failed, st = plan.exec_file(fin, fout, chunks, n_slots=3,
                                            io_threads=args.io_threads)
            tl = plan.stream_timeline()
        if rc != 0:
            raise RuntimeError("file run failed at chunk %s (status %d)" % (failed, rc))
        # Parseval on every segment of the first and last chunk
        dev = 0.0
        with open(fout, "rb") as f:
            for c in sorted({0, chunks - 1}):
                f.seek(c * chunk)
                y = np.frombuffer(f.read(chunk), np.complex64).reshape(seg, n)
                _, e_in = sig.segments_with_energy(c * seg, seg)
                dev = max(dev, float(np.max(np.abs(segment_energy(y) / (n * e_in) - 1.0))))
        import bench_profile
        H, K, D = bench_profile.timeline_intervals(tl)
        ov = bench_profile.overlap_stats(H, [iv for ks in K for iv in ks], D)
        wall = st["wall_s"]
        out = {"workload": "file_%s_4096pt" % ("%dGiB" % (size >> 30)),
               "file_bytes": size, "chunks": chunks, "chunk_bytes": chunk,
               "dir": d, "filesystem": _fs_type(d), "io_threads": args.io_threads,
               "input_write_s": round(t_write_in, 2),
               "wall_s": round(wall, 3),
               "end_to_end_GBps": round(size / wall / 1e9, 2),
               "file_read_GBps": round(size / max(st["fill_s"], 1e-9) / 1e9, 2),
               "file_write_GBps": round(size / max(st["drain_s"], 1e-9) / 1e9, 2),
               "read_s": round(st["fill_s"], 3), "write_s": round(st["drain_s"], 3),
               "h2d_GBps_per_copy": round(size / max(st["h2d_s"], 1e-9) / 1e9, 2),
               "d2h_GBps_per_copy": round(size / max(st["d2h_s"], 1e-9) / 1e9, 2),
               "transform_s": round(st["compute_s"], 4),
               "share_transform": round(st["compute_s"] / wall, 4),
               "share_file_io": round((st["fill_s"] + st["drain_s"]) / wall, 4),
               "device_idle_ms": round(ov["device_idle_ms"], 1),
               "paper_context": "GPU run: FFT 5-8 % of the time, I/O the rest; CPU run: "
                                "disk I/O 70-75 % (Sec. IV, Figs. 4-5)",
               "parseval_max_rel_dev_first_last_chunk": dev,
               "parseval_bound": 2 * 5e-7 * math.log2(n) + (5e-7 * math.log2(n)) ** 2}
        print(json.dumps(out), flush=True)
        return 0 if dev <= out["parseval_bound"] else 1
    finally:
        buf.close()
        for p in (fin, fout):
            try:
                os.remove(p)
            except OSError:
                pass


def run(args):
    return {"small": small, "uneven": uneven, "streamed": streamed,
            "serving": serving, "long": long, "real": real,
            "frames": frames, "file": file, "lengths": lengths,
            "frame_lengths": frame_lengths}[args.workload](args)
