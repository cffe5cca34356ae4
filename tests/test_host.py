"""Host-side logic that needs no device: the launch autotuner's walk (on a
stand-in handle), its JSON round trip, the benchmark's single-GPU guard and
the gate that keeps a stale HBM-traffic record out of the bench line."""
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


def test_tuned_options_name_known_options():
    import bench
    from paper_1702_04645_amd import autotune
    opts = bench.tuned_options("rmat20")
    assert opts and set(opts) <= set(autotune.CANDIDATES)
    assert bench.tuned_options("no_such_workload") is None
