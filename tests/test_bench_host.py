"""bench.py host logic (no GPU): the one-GPU rule and the recorded traffic of
the dominant kernel, which must be ignored once the kernel's sources change."""
import hashlib
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


def _sha(root, files):
    return hashlib.sha256(b"".join(open(os.path.join(root, f), "rb").read() for f in files)).hexdigest()


def test_recorded_traffic_follows_the_sources():
    """A record counts only while the kernel's sources hash to what it names."""
    recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, rec in recs.items():
        workload, schedule = key.rsplit("/", 1)
        want = (rec["fetch_kib_avg"] * rec["fetch_scale"] + rec["write_kib_avg"] * rec["write_scale"]) * 1024.0
        got = bench.recorded_traffic(workload, schedule)
        assert got == (want if _sha(ROOT, rec["sources"]) == rec["sources_sha256"] else None), key
    assert bench.recorded_traffic("no-such-workload", "hub") is None


def test_recorded_traffic_is_dropped_when_a_source_changes(tmp_path, monkeypatch):
    rec = {"kernel": "k", "sources": ["paper_2009_07929_amd/csrc/k_support.hip", "paper_2009_07929_amd/csrc/common.h"],
           "fetch_kib_avg": 100.0, "write_kib_avg": 10.0, "fetch_scale": 2.0, "write_scale": 1.0}
    for f in rec["sources"]:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), tmp_path / f)
    rec["sources_sha256"] = _sha(str(tmp_path), rec["sources"])
    (tmp_path / "profiles").mkdir()
    json.dump({"w/hub": rec}, open(tmp_path / "profiles" / "traffic.json", "w"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("w", "hub") == (100.0 * 2.0 + 10.0) * 1024.0
    assert bench.recorded_traffic("w", "plain") is None
    with open(tmp_path / rec["sources"][0], "a") as fh:
        fh.write("\n// edited\n")
    assert bench.recorded_traffic("w", "hub") is None
