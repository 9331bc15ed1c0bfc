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


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        kernels(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6:8])
    else:
        raise SystemExit(__doc__)
