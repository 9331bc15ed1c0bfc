"""Plans replayed as hipGraphs, and the autotuner with its JSON cache."""
import json

import numpy as np
import pytest

import oracle
import paper_1407_6915_amd as fs

from gpu_helpers import announce, noise

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,batch", [(4096, 300), (1 << 16, 5), (1 << 20, 2), (3 ** 9, 3), (1, 7)])
def test_plan_graph_replays_match_eager(n, batch):
    import torch
    announce("plan graph n=%d" % n)
    x = noise(n, batch, seed=21)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    eager = torch.empty_like(xd)
    outg = torch.empty_like(xd)
    sh = torch.cuda.current_stream().cuda_stream
    with fs.Plan(n, batch) as p:
        p.exec_ptr(xd.data_ptr(), eager.data_ptr(), sh)
        torch.cuda.synchronize()
        ref = eager.cpu().numpy()
        assert np.all(oracle.rel_l2(ref.reshape(batch, n), oracle.fft_recursive(x, n))
                      <= oracle.tolerance(n))
        for i in range(4):
            outg.fill_(float(i))                    # eager work between replays
            p.exec_graph_ptr(xd.data_ptr(), outg.data_ptr(), sh)
            torch.cuda.synchronize()
            assert np.array_equal(outg.cpu().numpy(), ref), i
        # new buffers -> re-capture
        out2 = torch.empty_like(xd)
        p.exec_graph_ptr(xd.data_ptr(), out2.data_ptr(), sh)
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy(), ref)


def test_autotune_and_cache(tmp_path):
    import torch
    announce("autotune 4096 x 8192")
    path = str(tmp_path / "tune.json")
    fs.tune_clear()
    k, best = fs.autotune(4096, 8192, fs.FORWARD, path)
    # every plan variant at 6 grids, then the work-list routes: the tiles
    # once, each indexed kernel at 6 grids
    assert k == fs.variant_count(4096) * 6 + 1 + 6 * fs.indexed_count(4096) and best > 0
    js = json.load(open(path))
    ent = [e for e in js["entries"] if e["n"] == 4096]
    assert len(ent) == 1 and 0 <= ent[0]["variant"] < fs.variant_count(4096)
    assert 0 <= ent[0]["wl_route"] <= fs.indexed_count(4096) and ent[0]["wl_us"] > 0
    assert js["arch"].startswith("gfx")
    # a work list built now takes the tuned route for its 4096-point segments
    ents = np.zeros(20, dtype=[("in_off", "<u8"), ("out_off", "<u8"),
                               ("segment_len", "<u4"), ("job", "<u4")])
    ents["in_off"] = ents["out_off"] = np.arange(20) * 4099
    ents["segment_len"] = 4096
    with fs.WorkList(ents) as wl:
        idx = wl.describe()["indexed"]
        if ent[0]["wl_route"] == 0:
            assert idx == {}
        else:
            assert idx["4096"]["candidate"] == ent[0]["wl_route"] - 1
    # a tuned plan reports the chosen variant and grid, and stays correct
    d = fs.Plan(4096, 64).describe()
    assert d["variant"] == ent[0]["variant"] and d["grid_mult"] == ent[0]["grid_mult"]
    x = noise(4096, 64, seed=2)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    with fs.Plan(4096, 64) as p:
        y = p.exec(xd).cpu().numpy().reshape(64, 4096)
    assert np.all(oracle.rel_l2(y, oracle.fft_recursive(x, 4096)) <= oracle.tolerance(4096))
    # two-pass lengths tune tile variants x grid and the split itself (the
    # planner's 256 x 256 and the other splits with tiles: 128 x 512,
    # 512 x 128); merged into the same file
    n1, n2, nc, nr = fs.split_info(1 << 16)
    k2, _ = fs.autotune(1 << 16, 64, fs.FORWARD, path)
    # plus the work-list routes: the tiles once, the indexed passes at 6 grids
    assert k2 == 6 * (nc * nr + 2) + 1 + 6 * fs.indexed_count(1 << 16)
    js = json.load(open(path))
    assert {e["n"] for e in js["entries"]} == {4096, 1 << 16}
    e2 = [e for e in js["entries"] if e["n"] == 1 << 16][0]
    assert e2["n1"] in (128, 256, 512)
    d2 = fs.Plan(1 << 16, 4).describe()
    assert d2["n1"] == e2["n1"] and d2["n1"] * d2["n2"] == 1 << 16
    assert d2["column_variant"] == e2["column_variant"]
    assert d2["row_variant"] == e2["row_variant"] and d2["grid_mult"] == e2["grid_mult"]
    x2 = noise(1 << 16, 4, seed=3)
    with fs.Plan(1 << 16, 4) as p2:
        y2 = p2.exec(torch.from_numpy(x2.reshape(-1)).cuda()).cpu().numpy().reshape(4, -1)
    assert np.all(oracle.rel_l2(y2, oracle.fft_recursive(x2, 1 << 16))
                  <= oracle.tolerance(1 << 16))
    fs.tune_clear()
    assert fs.Plan(4096, 64).describe()["variant"] == 0
    assert fs.tune_load(path) == 2
    assert fs.Plan(4096, 64).describe()["variant"] == ent[0]["variant"]
    fs.tune_clear()
