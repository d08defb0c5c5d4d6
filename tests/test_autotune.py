"""Autotuner host logic (no GPU): graph classes, tuning mapping, cache."""
import numpy as np

import synth
from paper_2009_07929_amd import autotune
from paper_2009_07929_amd import ktruss as kt


def test_graph_class_buckets():
    n, s, d = synth.rmat(12, 8, 0.57, 0.19, 0.19, 1)
    rp, col, _ = kt.ktruss_build_csr(s, d, n)
    c = autotune.graph_class(rp)
    assert c.startswith("m2^15-") and autotune.graph_class(rp) == c
    assert autotune.graph_class(np.zeros(5, np.int32)) == "m2^0-skew2^0"
    assert autotune.batch_class(4096, 2 ** 27) == "batch-G4096-m2^27"


def test_to_tuning_fields():
    cfg = dict(autotune.DEFAULT, hub_chunk_tasks=64, rounds_per_sync=4, learned_hub_min=12.5)
    t = autotune.to_tuning(cfg)
    assert t.hub_chunk_tasks == 64 and t.rounds_per_sync == 4 and abs(t.learned_hub_min - 12.5) < 1e-6
    assert t.wave_min_work == cfg["wave_min_work"] and t.hub_min_work == cfg["hub_min_work"]
    assert autotune.to_tuning(dict(cfg, plain_max_work=128)).plain_max_work == 128
    old = {k: v for k, v in cfg.items() if k != "plain_max_work"}   # entries cached before the gate existed
    assert autotune.to_tuning(old).plain_max_work == 0
    older = {k: v for k, v in old.items() if k not in ("incremental", "peel_ratio")}
    assert autotune.to_tuning(older).incremental == 0    # entries cached before incremental maintenance
    t = autotune.to_tuning(dict(cfg, incremental=2, peel_ratio=0.25))
    assert t.incremental == 2 and abs(t.peel_ratio - 0.25) < 1e-7


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "cache.json")
    assert autotune.tuned_config("x/K3", path) == autotune.DEFAULT
    cfg = dict(autotune.DEFAULT, schedule="heuristic")
    autotune.store("x/K3", cfg, 0.01, path)
    assert autotune.tuned_config("x/K3", path) == cfg
    assert autotune.load_cache(path)["x/K3"]["seconds"] == 0.01
