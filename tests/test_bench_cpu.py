"""Host-side logic of bench.py and bench_profile.py (no GPU needed)."""
import csv
import json
import os
import subprocess
import sys

import bench
import bench_profile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_scaling_against_the_copy_kernel(tmp_path):
    samples = 1 << 20
    known_kib = samples * 8 / 1024.0
    fft = "void fftseg::single_pass_plain_kernel<...>(...)"
    copy = "__amd_rocclr_copyBuffer"
    # FETCH_SIZE counts half of the bytes read, WRITE_SIZE all of them; the
    # transform reads 10 % more than it writes
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(copy, 0.5 * known_kib), (fft, 0.55 * known_kib), (fft, 0.55 * known_kib)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(copy, known_kib), (fft, known_kib)])
    out = tmp_path / "t.json"
    bench_profile.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out), samples,
                          ["cmd f", "cmd w"])
    d = json.load(open(out))
    assert abs(d["fetch_scale"] - 0.5) < 1e-12 and abs(d["write_scale"] - 1.0) < 1e-12
    assert abs(d["hbm_fetch_bytes_per_launch"] - 1.1 * samples * 8) < 1e-3
    assert abs(d["hbm_write_bytes_per_launch"] - samples * 8) < 1e-3
    assert abs(d["traffic_over_algorithmic"] - 2.1 / 2.0) < 1e-12
    assert d["commands"] == ["cmd f", "cmd w"]
    assert d["kernel_source_hash"] == bench.kernel_source_hash()


def test_traffic_is_reported_only_for_the_measured_kernel(tmp_path, monkeypatch):
    rec = {"kernel_source_hash": bench.kernel_source_hash(), "samples_per_launch": 4096,
           "hbm_bytes_per_launch": 123.0}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic(4096) == 123.0
    assert bench.measured_traffic(8192) is None          # another workload size
    rec["kernel_source_hash"] = "0" * 16                  # another kernel
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(4096) is None


def test_overlap_summary_from_traces(tmp_path):
    """Two chunks: H2D 0-10 / 10-20 ms, transforms 10-14 / 20-24, D2H
    14-24 / 24-34 (ms); small copies are ignored."""
    ms = 1_000_000
    kp, cp = tmp_path / "k.csv", tmp_path / "c.csv"
    with open(kp, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for a, b in [(10, 12), (12, 14), (20, 22), (22, 24)]:
            w.writerow({"Kernel_Name": "four_step_columns_kernel<...>",
                        "Start_Timestamp": a * ms, "End_Timestamp": b * ms})
        w.writerow({"Kernel_Name": "other", "Start_Timestamp": 0, "End_Timestamp": 50 * ms})
    with open(cp, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Direction", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        rows = [("MEMORY_COPY_HOST_TO_DEVICE", 0, 10), ("MEMORY_COPY_HOST_TO_DEVICE", 10, 20),
                ("MEMORY_COPY_DEVICE_TO_HOST", 14, 24), ("MEMORY_COPY_DEVICE_TO_HOST", 24, 34)]
        for d, a, b in rows:
            w.writerow({"Direction": d, "Start_Timestamp": a * ms, "End_Timestamp": b * ms})
        w.writerow({"Direction": "MEMORY_COPY_HOST_TO_DEVICE", "Start_Timestamp": 40 * ms,
                    "End_Timestamp": 40 * ms + 1000})
    out = tmp_path / "o.md"
    bench_profile.overlap(str(kp), str(cp), str(out), 2, "cmd")
    text = out.read_text()
    assert "| 0 | 0.0–10.0 | 10.0–14.0 | 14.0–24.0 |" in text
    assert "| 1 | 10.0–20.0 | 20.0–24.0 | 24.0–34.0 |" in text
    assert "wall (first H2D start to last D2H end): 34.0 ms" in text
    # busy 20 + 20 + 8 = 48 ms over 34 ms of wall
    assert "sum of busy intervals / wall: 1.41" in text
    # transforms 10-14 (H2D 10-20 in flight) and 20-24 (D2H 14-24 in flight)
    assert "transform time with a copy in flight: 100.0 %" in text
    # H2D 10-20 overlaps D2H 14-24 for 6 of the 20 ms
    assert "H2D time with a D2H in flight: 30.0 %" in text
    assert "device idle (no copy and no transform): 0.0 ms" in text


def test_traffic_table_per_sample(tmp_path):
    copy_samples = 1 << 20
    known_kib = copy_samples * 8 / 1024
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    # FETCH_SIZE counts half of the bytes read, WRITE_SIZE all of them
    _counter_csv(fp, "FETCH_SIZE", [("identity_copy_kernel<x>", known_kib / 2),
                                    ("four_step_columns_kernel<a>", known_kib / 2 / 4),
                                    ("four_step_columns_kernel<a>", known_kib / 2 / 4),
                                    ("single_pass_plain_kernel<b>", known_kib / 2 * 1.5)])
    _counter_csv(wp, "WRITE_SIZE", [("identity_copy_kernel<x>", known_kib),
                                    ("four_step_columns_kernel<a>", known_kib / 4),
                                    ("four_step_columns_kernel<a>", known_kib / 4),
                                    ("single_pass_plain_kernel<b>", known_kib)])
    out = tmp_path / "t.json"
    bench_profile.traffic_table(str(fp), str(wp), str(out), copy_samples,
                                [("four_step", copy_samples // 4),
                                 ("single_pass", copy_samples)])
    t = json.load(open(out))
    rows = {r["kernel"]: r for r in t["kernels"]}
    col = rows["four_step_columns_kernel<a>"]
    assert col["dispatches"] == 2
    assert abs(col["hbm_read_bytes_per_sample"] - 8.0) < 1e-9
    assert abs(col["hbm_write_bytes_per_sample"] - 8.0) < 1e-9
    sp = rows["single_pass_plain_kernel<b>"]
    assert abs(sp["hbm_read_bytes_per_sample"] - 12.0) < 1e-9
    assert abs(sp["hbm_bytes_per_sample"] - 20.0) < 1e-9
