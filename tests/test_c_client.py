"""The C ABI from a C program (tests/c_client/stream_client.c): it compiles
and links against libfftseg.so with gcc on any host; on a GPU it streams
chunks of impulses through the pipeline and checks their spectra."""
import json
import os
import subprocess

import pytest

import paper_1407_6915_amd as fs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_client", "stream_client.c")


def build_client(out_path):
    lib_dir = os.path.dirname(fs.LIB_PATH)
    if not os.path.exists(fs.LIB_PATH):
        fs.build()
    cmd = ["gcc", "-O2", "-Wall", "-Wextra", "-Werror", "-std=c11",
           "-I" + os.path.join(ROOT, "include"), SRC, "-L" + lib_dir, "-lfftseg",
           "-Wl,-rpath," + lib_dir, "-o", str(out_path)]
    subprocess.check_call(cmd)
    return str(out_path)


def test_client_builds(tmp_path):
    exe = build_client(tmp_path / "stream_client")
    assert os.access(exe, os.X_OK)
    # wrong argument counts and values are refused before any device work
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
    r = subprocess.run([exe, "4096", "0", "1", "1"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2


@pytest.mark.gpu
def test_client_streams_on_the_gpu(tmp_path):
    from gpu_helpers import announce
    announce("C client: 4096 x 1024 per chunk, 6 chunks, pool of 2")
    exe = build_client(tmp_path / "stream_client")
    r = subprocess.run([exe, "4096", "1024", "6", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    tl = out["timeline_ms"]
    assert [t[0] for t in tl] == list(range(6))
    for t in tl:
        assert all(a <= b for a, b in zip(t[1:], t[2:])), t
