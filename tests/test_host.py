"""Host-side logic that needs no device: the launch autotuner's walk (on a
stand-in handle), its JSON round trip, its cache keyed by GPU architecture
and degree profile, the benchmark's single-GPU guard and the gate that keeps
a stale HBM-traffic record out of the bench line."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


class _Arr:
    def __init__(self, a):
        self.a = a

    def cpu(self):
        return self

    def numpy(self):
        return self.a


class _FakeGraph:
    """Sweeps whose time depends on the options: grid_512 = 512 and
    hub_table_bits = 10 are fastest; 'bad' makes an option change the output."""

    def __init__(self, bad=None):
        self.opt = {}
        self.bad = bad
        self.sweeps = 0

    def set_option(self, k, v):
        self.opt[k] = v

    def sweep(self, lab, nc):
        self.sweeps += 1
        out = np.arange(8, dtype=np.int32)
        if self.bad and self.opt.get(self.bad[0]) == self.bad[1]:
            out = out + 1
        return _Arr(out), _Arr(np.zeros(8, np.int64)), _Arr(np.ones(8, np.int32))

    def timing(self, on):
        self.sweeps = 0

    def timing_read(self):
        us = 100.0
        if self.opt.get("grid_512") == 512:
            us -= 10
        if self.opt.get("hub_table_bits") == 10:
            us -= 5
        n, self.sweeps = self.sweeps, 0
        return {"sweep_ms": us * n / 1e3, "sweeps": n}


@pytest.fixture
def no_cuda_sync(monkeypatch):
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def test_autotune_walk_and_round_trip(tmp_path, no_cuda_sync):
    from paper_1702_04645_amd import autotune
    g = _FakeGraph()
    res = autotune.tune(g, lab=np.zeros(8), nc=8, reps=2, blocks=1, passes=2)
    assert res["options"]["grid_512"] == 512
    assert res["options"]["hub_table_bits"] == 10
    assert res["us"] == pytest.approx(85.0) and res["us_default"] == pytest.approx(100.0)
    for k, v in res["options"].items():
        assert v in autotune.CANDIDATES[k]
    path = tmp_path / "t.json"
    autotune.save(path, res)
    assert autotune.load(path) == json.loads(json.dumps(res))
    g2 = _FakeGraph()
    autotune.apply(g2, res["options"])
    assert g2.opt == res["options"]


def test_autotune_refuses_an_option_that_changes_the_sweep(no_cuda_sync):
    from paper_1702_04645_amd import autotune
    with pytest.raises(AssertionError):
        autotune.tune(_FakeGraph(bad=("grid_256", 1024)), lab=np.zeros(8), nc=8, reps=1,
                      blocks=1, passes=1)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_is_gated_on_the_sweep_sources(monkeypatch):
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "rmat20_sweep_hbm_traffic.json")))
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: rec["sweep_source_sha256_16"])
    assert bench.measured_traffic("rmat20") == round(rec["sweep_traffic_bytes"] / 1e9, 4)
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("rmat20") is None
    assert bench.measured_traffic("no_such_workload") is None


def test_degree_profile():
    from paper_1702_04645_amd import autotune
    # degrees 0, 3, 2, 0, 100: 5 entries in the bin of rows up to 8, 100 in
    # the bin of rows of 65..128
    p = autotune.degree_profile(np.array([0, 0, 3, 5, 5, 105]))
    assert p == {"entries_log2": 7, "bin_shares": [0, 1, 0, 0, 19, 0, 0, 0, 0, 0, 0]}
    # a bin's upper limit belongs to it; a row above 4096 is a hub
    p = autotune.degree_profile(np.array([0, 8, 16, 4112]))
    assert p["bin_shares"] == [0, 0, 0, 0, 0, 0, 0, 0, 0, 20, 0]
    p = autotune.degree_profile(np.array([0, 8, 16, 4113]))
    assert p["bin_shares"] == [0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 20]
    p = autotune.degree_profile(np.array([0, 8, 16]))
    assert p["bin_shares"] == [0, 20, 0, 0, 0, 0, 0, 0, 0, 0, 0]
    assert autotune.degree_profile(np.array([0, 0]))["entries_log2"] == 0
    assert autotune.profile_key(np.array([0, 8, 16]), "gfx950") == "gfx950|e4|0,20,0,0,0,0,0,0,0,0,0"


def test_kept_tuned_files_are_keyed():
    from paper_1702_04645_amd import autotune
    d = os.path.join(ROOT, "paper_1702_04645_amd", "tuned")
    names = sorted(os.listdir(d))
    assert names
    for name in names:
        rec = autotune.load(os.path.join(d, name))
        assert autotune.cache_path(rec["key"], d) == os.path.join(d, name)
        p = rec["profile"]
        assert rec["key"] == "%s|e%d|%s" % (rec["arch"], p["entries_log2"],
                                           ",".join(str(x) for x in p["bin_shares"]))
        assert set(rec["options"]) == set(autotune.CANDIDATES)
        for k, v in rec["options"].items():
            assert v in autotune.CANDIDATES[k]


def test_tuned_options_are_keyed_by_device_and_degree_profile(tmp_path, monkeypatch):
    import bench
    import graphgen as gg
    from paper_1702_04645_amd import autotune
    monkeypatch.delenv("SLM_TUNE_CACHE", raising=False)
    rp = gg.config_graph("rmat20")[0]
    opts, path = bench.tuned_options(rp, arch="gfx950")
    assert opts and set(opts) <= set(autotune.CANDIDATES)
    assert autotune.load(path)["workload"] == "rmat20"
    assert bench.tuned_options(rp, arch="gfx942") == (None, None)
    small = gg.config_graph("sbm4096")[0]
    assert bench.tuned_options(small, arch="gfx950") == (None, None)
    # a cache folder of the caller's: SLM_TUNE_CACHE
    monkeypatch.setenv("SLM_TUNE_CACHE", str(tmp_path))
    assert bench.tuned_options(rp, arch="gfx950") == (None, None)
    res = {"options": dict(autotune.DEFAULTS, grid_512=512), "us": 1.0, "us_default": 2.0}
    p = autotune.save_keyed(small, "gfx950", res, workload="sbm4096")
    assert os.path.dirname(p) == str(tmp_path)
    assert bench.tuned_options(small, arch="gfx950") == (res["options"], p)
    # a file whose key is not the graph's is not used
    rec = autotune.load(p)
    rec["key"] = rec["key"] + ",0"
    autotune.save(p, rec)
    assert autotune.find(small, "gfx950") == (None, None)
    # an unreadable cache leaves the library defaults
    with open(p, "w") as f:
        f.write("{")
    assert bench.tuned_options(small, arch="gfx950") == (None, None)
