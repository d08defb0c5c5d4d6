"""bench.py host logic (no GPU): the one-GPU rule and the recorded traffic of
the dominant kernel, which must be ignored once the kernel's sources change."""
import json
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_recorded_traffic_matches_the_committed_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["rmat-s20-ef16/hub"]
    want = (rec["fetch_kib_avg"] * rec["fetch_scale"] + rec["write_kib_avg"] * rec["write_scale"]) * 1024.0
    assert bench.recorded_traffic("rmat-s20-ef16", "hub") == want
    assert bench.recorded_traffic("rmat-s20-ef16", "plain") is None
    assert bench.recorded_traffic("no-such-workload", "hub") is None


def test_recorded_traffic_is_dropped_when_a_source_changes(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    (tmp_path / "profiles").mkdir()
    json.dump(rec, open(tmp_path / "profiles" / "traffic.json", "w"))
    for f in rec["rmat-s20-ef16/hub"]["sources"]:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), tmp_path / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("rmat-s20-ef16", "hub") is not None
    with open(tmp_path / rec["rmat-s20-ef16/hub"]["sources"][0], "a") as fh:
        fh.write("\n// edited\n")
    assert bench.recorded_traffic("rmat-s20-ef16", "hub") is None
