#!/usr/bin/env python3
"""Turn rocprofv3 CSV output of ``bench.py`` runs into the summaries kept
under profiles/.

  kernels  <kernel_stats.csv> <out.md> <command...>
           per-kernel call count and average/min/max duration
  traffic  <fetch counter_collection.csv> <write counter_collection.csv>
           <out.json> <samples per launch> [<fetch command> <write command>]
           HBM bytes per launch of the transform kernel, from FETCH_SIZE and
           WRITE_SIZE (KiB per dispatch), each scaled by what the same counter
           reads for the plain device copy of a known size in the same run
           (bench.py --copy-reference copies samples*8 bytes each way)

  traffic_table <fetch.csv> <write.csv> <out.json> <copy samples> <pattern=samples>...
           [-- <fetch command> <write command>]
           HBM bytes per sample of every kernel whose name contains a
           pattern (samples per dispatch given per pattern), scaled by the
           same counters on identity_copy_kernel of copy samples * 8 bytes
  counters <counter_collection.csv> <out.md> <command...>
           per-kernel means of every counter of one --pmc run and the
           conflict and wait ratios
  overlap  <kernel_trace.csv> <memory_copy_trace.csv> <out.md> <chunks> <command...>
           per-chunk host-to-device copy, transform and device-to-host copy
           intervals of the streamed runs (bench.py --workload streamed), and
           how much of the time copies and transforms overlap

The traffic file records the hash of the device sources it was measured
on; bench.py reports it only while the sources are unchanged.
"""
from __future__ import annotations

import csv
import json
import sys

import bench


def _short(name: str) -> str:
    name = name.strip('"')
    if name.startswith("void "):
        name = name[5:]
    return name if len(name) < 400 else name[:397] + "..."


def kernels(stats_csv: str, out_md: str, command: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# Kernel time summary", "", "Command (run from the repository root):", "",
             "    " + command, "",
             "| kernel | calls | avg us | min us | max us | share |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %.1f%% |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(counter_csv: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    out = {}
    for r in csv.DictReader(open(counter_csv)):
        if r.get("Counter_Name", counter) != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _is_fft(name: str) -> bool:
    return "single_pass_kernel" in name or "single_pass_plain_kernel" in name


def _split(per_kernel):
    fft = {k: v for k, v in per_kernel.items() if _is_fft(k)}
    copy = {k: v for k, v in per_kernel.items()
            if not _is_fft(k) and ("copy" in k.lower() or "elementwise" in k.lower())}
    if len(fft) != 1 or not copy:
        raise SystemExit("expected one transform kernel and a copy kernel, got %s"
                         % sorted(per_kernel))
    (fk, fv), = fft.items()
    ck = max(copy, key=lambda k: max(copy[k]))
    return fk, fv, ck, copy[ck]


def traffic(fetch_csv: str, write_csv: str, out_json: str, samples: int,
            commands=()) -> None:
    known = samples * 8.0                      # bytes the copy reads, and writes
    f_name, f_fft, c_name, f_copy = _split(_per_kernel(fetch_csv, "FETCH_SIZE"))
    _, w_fft, _, w_copy = _split(_per_kernel(write_csv, "WRITE_SIZE"))
    mean = lambda v: sum(v) / len(v)           # noqa: E731
    f_scale = mean(f_copy) * 1024.0 / known    # counter bytes per real byte
    w_scale = mean(w_copy) * 1024.0 / known
    fetch = mean(f_fft) * 1024.0 / f_scale
    write = mean(w_fft) * 1024.0 / w_scale
    out = {
        "kernel": _short(f_name),
        "copy_kernel": _short(c_name),
        "samples_per_launch": samples,
        "algorithmic_bytes_per_launch": 16.0 * samples,
        "fetch_KiB_per_dispatch": mean(f_fft), "write_KiB_per_dispatch": mean(w_fft),
        "copy_fetch_KiB": mean(f_copy), "copy_write_KiB": mean(w_copy),
        "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_fetch_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
        "hbm_bytes_per_launch": fetch + write,
        "traffic_over_algorithmic": (fetch + write) / (16.0 * samples),
        "kernel_source_hash": bench.kernel_source_hash(),
        "commands": list(commands),
    }
    json.dump(out, open(out_json, "w"), indent=1)
    print(json.dumps(out))


def traffic_table(fetch_csv: str, write_csv: str, out_json: str, copy_samples: int,
                  samples_rules, commands=()) -> None:
    """HBM bytes per sample of every kernel in the two counter runs, scaled
    by what FETCH_SIZE / WRITE_SIZE read for identity_copy_kernel, which
    moves copy_samples * 8 bytes each way per dispatch.  samples_rules:
    [(substring of the kernel name, samples per dispatch)], first match
    wins."""
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    mean = lambda v: sum(v) / len(v)           # noqa: E731
    copy = [k for k in fetch if "identity_copy_kernel" in k]
    if len(copy) != 1:
        raise SystemExit("expected one identity_copy_kernel, got %s" % copy)
    known = copy_samples * 8.0
    f_scale = mean(fetch[copy[0]]) * 1024.0 / known
    w_scale = mean(write[copy[0]]) * 1024.0 / known
    rows = []
    for k in sorted(fetch):
        if k not in write or k == copy[0]:
            continue
        samples = next((sp for pat, sp in samples_rules if pat in k), None)
        if samples is None:
            continue
        fb = mean(fetch[k]) * 1024.0 / f_scale
        wb = mean(write[k]) * 1024.0 / w_scale
        rows.append({"kernel": _short(k), "dispatches": len(fetch[k]),
                     "samples_per_dispatch": samples,
                     "fetch_KiB_per_dispatch": mean(fetch[k]),
                     "write_KiB_per_dispatch": mean(write[k]),
                     "hbm_read_bytes_per_sample": fb / samples,
                     "hbm_write_bytes_per_sample": wb / samples,
                     "hbm_bytes_per_sample": (fb + wb) / samples,
                     "algorithmic_bytes_per_sample": 16.0})
    out = {"copy_kernel": _short(copy[0]), "copy_bytes_each_way": known,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": rows,
           "commands": list(commands)}
    json.dump(out, open(out_json, "w"), indent=1)
    print(json.dumps(out, indent=1))


def counters(counter_csv: str, out_md: str, command: str) -> None:
    """Per-kernel means of every counter in one --pmc run, plus the derived
    ratios used to read them: LDS bank-conflict cycles per LDS instruction,
    and the share of wave cycles spent waiting (SQ_WAIT_ANY) and waiting
    to issue (SQ_WAIT_INST_ANY)."""
    per = {}
    for r in csv.DictReader(open(counter_csv)):
        d = per.setdefault(r["Kernel_Name"], {"vgpr": r.get("VGPR_Count", ""),
                                             "lds": r.get("LDS_Block_Size", ""),
                                             "wg": r.get("Workgroup_Size", "")})
        d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for d in per.values() for c in d if c not in ("vgpr", "lds", "wg")})
    lines = ["# Counters per kernel", "", "Command (run from the repository root):", "",
             "    " + command, "",
             "Means over each kernel's dispatches.  conflict/LDS = SQ_LDS_BANK_CONFLICT / "
             "SQ_INSTS_LDS; wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES; issue wait = "
             "SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES.", "",
             "| kernel | workgroup | VGPRs | LDS bytes | " + " | ".join(names) +
             " | conflict/LDS | wait | issue wait |",
             "|---|---|---|---|" + "---|" * len(names) + "---|---|---|"]
    for k, d in per.items():
        if k.startswith("__amd") or "at::native" in k:
            continue
        m = {c: sum(d[c]) / len(d[c]) for c in names if c in d}
        ratio = lambda a, b: ("%.2f" % (m[a] / m[b])) if m.get(b) else "—"  # noqa: E731
        lines.append("| `%s` | %s | %s | %s | " % (_short(k)[:150], d["wg"], d["vgpr"], d["lds"]) +
                     " | ".join("%.3g" % m[c] if c in m else "—" for c in names) + " | " +
                     " | ".join([ratio("SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS"),
                                 ratio("SQ_WAIT_ANY", "SQ_WAVE_CYCLES"),
                                 ratio("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")]) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError("none of %s in %s" % (names, sorted(row)))


def _union(iv):
    """Total length covered by a list of (start, end) intervals."""
    tot, cur_s, cur_e = 0.0, None, None
    for a, b in sorted(iv):
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot


def _covered(iv, by):
    """Length of the intervals iv that lies inside the union of `by`."""
    tot = 0.0
    merged = []
    for a, b in sorted(by):
        if merged and a <= merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], b)
        else:
            merged.append([a, b])
    for a, b in iv:
        for c, d in merged:
            lo, hi = max(a, c), min(b, d)
            if hi > lo:
                tot += hi - lo
    return tot


def overlap_stats(H, K, D):
    """Overlap figures of one streamed run from its chunk intervals: H (copy
    in), K (transforms), D (copy out), each a list of (start, end) in ns."""
    t0, t1 = min(a for a, _ in H), max(b for _, b in D)
    wall = t1 - t0
    sum_h = sum(b - a for a, b in H)
    sum_d = sum(b - a for a, b in D)
    sum_k = sum(b - a for a, b in K)
    return {"wall_ms": wall / 1e6, "h2d_busy_ms": sum_h / 1e6, "d2h_busy_ms": sum_d / 1e6,
            "transform_busy_ms": sum_k / 1e6,
            "busy_over_wall": (sum_h + sum_d + sum_k) / wall,
            "device_idle_ms": (wall - _union(H + D + K)) / 1e6,
            "transform_with_copy_in_flight": _covered(K, H + D) / max(sum_k, 1),
            "h2d_with_d2h_in_flight": _covered(H, D) / max(sum_h, 1)}


def overlap_lines(title, H, K_per_chunk, D, chunk_bytes):
    """Markdown table and figures of one run (intervals in ns)."""
    K = [iv for ks in K_per_chunk for iv in ks]
    st = overlap_stats(H, K, D)
    t0 = min(a for a, _ in H)
    ms = lambda t: (t - t0) / 1e6  # noqa: E731
    lines = ["## " + title, "",
             "| chunk | H2D start–end | transform start–end | D2H start–end |",
             "|---|---|---|---|"]
    for c in range(len(H)):
        kc = K_per_chunk[c]
        ks = "%.1f–%.1f" % (ms(kc[0][0]), ms(kc[-1][1])) if kc else "—"
        lines.append("| %d | %.1f–%.1f | %s | %.1f–%.1f |" % (
            c, ms(H[c][0]), ms(H[c][1]), ks, ms(D[c][0]), ms(D[c][1])))
    n = len(H)
    lines += ["",
              "* wall (first H2D start to last D2H end): %.1f ms" % st["wall_ms"],
              "* H2D busy %.1f ms (%.1f GB/s per copy), D2H busy %.1f ms (%.1f GB/s per "
              "copy), transforms %.1f ms" % (
                  st["h2d_busy_ms"], n * chunk_bytes / st["h2d_busy_ms"] / 1e6,
                  st["d2h_busy_ms"], n * chunk_bytes / st["d2h_busy_ms"] / 1e6,
                  st["transform_busy_ms"]),
              "* sum of busy intervals / wall: %.2f (1.0 would mean no overlap)"
              % st["busy_over_wall"],
              "* device idle (no copy and no transform): %.1f ms of %.1f" % (
                  st["device_idle_ms"], st["wall_ms"]),
              "* transform time with a copy in flight: %.1f %%" % (
                  100.0 * st["transform_with_copy_in_flight"]),
              "* H2D time with a D2H in flight: %.1f %%" % (100.0 * st["h2d_with_d2h_in_flight"]),
              ""]
    return lines


def timeline_intervals(timeline):
    """(H, K per chunk, D) in ns from fft_stream_last_timeline entries."""
    ns = lambda v: int(round(v * 1e6))  # noqa: E731
    H = [(ns(t["h2d_start_ms"]), ns(t["h2d_end_ms"])) for t in timeline]
    K = [[(ns(t["compute_start_ms"]), ns(t["compute_end_ms"]))] for t in timeline]
    D = [(ns(t["d2h_start_ms"]), ns(t["d2h_end_ms"])) for t in timeline]
    return H, K, D


def overlap(kernel_csv: str, copy_csv: str, out_md: str, chunks: int, command: str) -> None:
    kern = []
    for r in csv.DictReader(open(kernel_csv)):
        name = _col(r, "Kernel_Name")
        if "four_step" in name:
            kern.append((int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp")), name))
    h2d, d2h = [], []
    for r in csv.DictReader(open(copy_csv)):
        a, b = int(_col(r, "Start_Timestamp")), int(_col(r, "End_Timestamp"))
        direction = _col(r, "Direction", "Operation", "Kind").upper()
        if b - a < 5_000_000:          # the chunk copies take tens of ms; skip small ones
            continue
        if "HOST_TO_DEVICE" in direction:
            h2d.append((a, b))
        elif "DEVICE_TO_HOST" in direction:
            d2h.append((a, b))
    h2d.sort()
    d2h.sort()
    kern.sort()
    runs = len(h2d) // chunks
    if runs == 0 or len(d2h) < runs * chunks:
        raise SystemExit("expected %d-chunk runs, got %d H2D and %d D2H chunk copies"
                         % (chunks, len(h2d), len(d2h)))
    names = ["pool of pre-generated pinned chunks (link reference)",
             "every chunk generated from the seed (as configured)"]
    lines = ["# Streamed 2^20-point chunks: copy/compute overlap", "",
             "Command (run from the repository root):", "", "    " + command, "",
             "Chunks of 512 segments (4 GiB each way). Intervals from the rocprofv3 kernel "
             "trace (the four-step column and row kernels of each chunk) and memory-copy "
             "trace (copies of 5 ms or more: the chunk copies), in ms from the run's "
             "first copy.", ""]
    for r in range(runs):
        H = h2d[r * chunks:(r + 1) * chunks]
        D = d2h[r * chunks:(r + 1) * chunks]
        t0, t1 = H[0][0], D[-1][1]
        K = [(a, b) for a, b, _ in kern if a >= t0 and b <= t1]
        per = [[(a, b) for a, b in K if a >= H[c][1] and b <= D[c][0]] for c in range(chunks)]
        title = "Run %d: %s" % (r + 1, names[r] if r < len(names) else "run %d" % (r + 1))
        lines += overlap_lines(title, H, per, D, 4 * 2 ** 30)
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        kernels(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6:8])
    elif sys.argv[1] == "traffic_table":
        # fetch.csv write.csv out.json copy_samples pattern=samples ... -- commands
        args = sys.argv[2:]
        cmds = args[args.index("--") + 1:] if "--" in args else []
        args = args[:args.index("--")] if "--" in args else args
        rules = [(a.split("=", 1)[0], int(a.split("=", 1)[1])) for a in args[4:]]
        traffic_table(args[0], args[1], args[2], int(args[3]), rules, cmds)
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "overlap":
        overlap(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), " ".join(sys.argv[6:]))
    else:
        raise SystemExit(__doc__)
