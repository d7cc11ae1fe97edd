"""Host-side checks of bench.py (no GPU needed): it refuses more than one GPU
before touching the device, and it reads HBM traffic from the committed
counter summary only while the kernel sources match it."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_follows_the_source_hash(monkeypatch):
    p = os.path.join(ROOT, "profiles", "traffic_4k_x8.json")
    t = json.load(open(p))
    ent = t["kernels"]["search_exhaustive_fused"]["hbm_bytes_per_launch"]
    assert ent > 0
    # the committed summary is used only while the sources hash to its value
    got = bench._traffic("search_exhaustive_fused")
    if t["source_hash"] == bench._kernel_source_hash():
        assert got == ent
    else:
        assert got is None
    # a summary taken from other sources is ignored
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "0" * 16)
    assert bench._traffic("search_exhaustive_fused") is None
    assert bench._traffic("no_such_kernel") is None
