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
