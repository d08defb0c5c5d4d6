"""Autotuner of the support schedule and its tile parameters.

Searches, by timed runs on the device, the schedule (hub, heuristic, learned,
plain) and the knobs of ktruss_tuning: tasks per hub item, the hub-row
threshold of the heuristic, the wavefront/thread cut-off, the learned
threshold, the light-graph gate, the number of prune rounds replayed from a
hipGraph per host check, and recompute vs incremental support maintenance
(with its peel ratio).  Results are
keyed by (graph class, K) and cached in a JSON file; a cached entry is reused
for any graph of the same class.  Every candidate produces identical results
(the schedule never changes the truss), so only time is compared.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import ktruss as kt

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")

SCHEDULE_IDS = {"plain": kt.SCHED_PLAIN, "heuristic": kt.SCHED_HEURISTIC, "learned": kt.SCHED_LEARNED,
                "hub": kt.SCHED_FORCE_HUB}

DEFAULT = {"schedule": "hub", "hub_chunk_tasks": 256, "hub_min_work": 8, "wave_min_work": 192,
           "hub_chunk_work": 0, "learned_hub_min": 0.0, "rounds_per_sync": 0, "plain_max_work": 0,
           "incremental": 2, "peel_ratio": 0.125}

# values tried per knob (coordinate search, in this order)
SPACE = [
    ("schedule", ["hub", "heuristic", "learned", "plain"]),
    ("hub_chunk_tasks", [64, 128, 256]),
    ("rounds_per_sync", [0, 4, 16]),
    ("hub_min_work", [2, 8, 32]),
    ("wave_min_work", [64, 192, 768]),
    ("learned_hub_min", [-0.5, 0.0, 0.5]),
    ("plain_max_work", [-1, 0, 128]),
    ("incremental", [0, 1, 2]),
    ("peel_ratio", [0.03125, 0.125, 0.5, 2.0]),
]
# knobs that only matter under some schedules
RELEVANT = {"hub_min_work": {"heuristic"}, "wave_min_work": {"heuristic", "learned"},
            "learned_hub_min": {"learned"}, "hub_chunk_tasks": {"hub", "heuristic", "learned"},
            "plain_max_work": {"heuristic", "learned"}, "rounds_per_sync": {"hub", "heuristic", "learned", "plain"}}


def graph_class(rowptr) -> str:
    """Size and skew buckets: log2 of the edge count and of max/mean row length."""
    rowptr = np.asarray(rowptr, np.int64)
    d = np.diff(rowptr)
    m = int(rowptr[-1])
    nz = d[d > 0]
    skew = float(nz.max()) / float(nz.mean()) if len(nz) else 1.0
    return "m2^%d-skew2^%d" % (int(round(math.log2(max(m, 1)))), int(round(math.log2(max(skew, 1.0)))))


def batch_class(G: int, m_total: int) -> str:
    return "batch-G%d-m2^%d" % (G, int(round(math.log2(max(m_total, 1)))))


def to_tuning(cfg) -> kt.ktruss_tuning:
    t = kt.ktruss_tuning()
    t.hub_chunk_tasks = int(cfg["hub_chunk_tasks"])
    t.hub_min_work = int(cfg["hub_min_work"])
    t.wave_min_work = int(cfg["wave_min_work"])
    t.learned_hub_min = float(cfg["learned_hub_min"])
    t.rounds_per_sync = int(cfg["rounds_per_sync"])
    t.plain_max_work = int(cfg.get("plain_max_work", 0))
    t.incremental = int(cfg.get("incremental", 0))   # entries cached before incremental maintenance: recompute
    t.peel_ratio = float(cfg.get("peel_ratio", 0.0))
    return t


def apply(target, cfg, mlp_params=None):
    """Set schedule and tuning on a Graph or Batch."""
    sched = SCHEDULE_IDS[cfg["schedule"]]
    if sched == kt.SCHED_LEARNED and mlp_params is None:
        sched = kt.SCHED_HEURISTIC
    if isinstance(target, kt.Batch):
        target.c.schedule = sched if sched != kt.SCHED_LEARNED else kt.SCHED_HEURISTIC
        target.c.tuning = to_tuning(cfg)
    else:
        kt.ktruss_set_schedule(target, sched, mlp_params, to_tuning(cfg))


def _timer(run, reps):
    import torch
    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def search(target, run, mlp_params=None, reps=3, sweeps=1, log=None):
    """Coordinate search from DEFAULT; `run()` executes one timed unit of work
    on `target` with whatever configuration was applied.  Returns (best cfg,
    best seconds, list of (cfg, seconds))."""
    best = dict(DEFAULT)
    if mlp_params is None:
        space = [(k, [v for v in vals if v != "learned"]) for k, vals in SPACE]
    else:
        space = SPACE
    if isinstance(target, kt.Batch):   # the batched form has no learned schedule
        space = [(k, [v for v in vals if v != "learned"]) for k, vals in space]
    apply(target, best, mlp_params)
    best_t = _timer(run, reps)
    trials = [(dict(best), best_t)]
    for _ in range(sweeps):
        for knob, values in space:
            if knob in RELEVANT and best["schedule"] not in RELEVANT[knob]:
                continue
            if knob == "peel_ratio" and best["incremental"] != 2:
                continue
            for v in values:
                if v == best[knob]:
                    continue
                cfg = dict(best)
                cfg[knob] = v
                apply(target, cfg, mlp_params)
                t = _timer(run, reps)
                trials.append((cfg, t))
                if log:
                    log("autotune %s=%s: %.3f ms (best %.3f ms)" % (knob, v, t * 1e3, best_t * 1e3))
                if t < best_t:
                    best, best_t = cfg, t
    apply(target, best, mlp_params)
    return best, best_t, trials


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def store(key, cfg, seconds, path=CACHE):
    data = load_cache(path)
    data[key] = {"config": cfg, "seconds": seconds}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_config(key, path=CACHE):
    """The cached configuration for `key`, or DEFAULT."""
    ent = load_cache(path).get(key)
    return dict(ent["config"]) if ent else dict(DEFAULT)


def tune_graph(g, K, mlp_params=None, reps=3, path=CACHE, log=None, rowptr=None):
    """Tune one graph for one K and store it under (graph class, K)."""
    import torch
    rp = rowptr if rowptr is not None else g.rowptr.cpu().numpy()
    key = "%s/K%d" % (graph_class(rp), K)
    mask = torch.empty(max(g.m, 1), dtype=torch.uint8, device=g.device)
    sup = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.device)
    best, t, _ = search(g, lambda: kt.ktruss_run(g, K, mask, sup), mlp_params, reps=reps, log=log)
    store(key, best, t, path)
    return key, best, t


def tune_batch(b, K_dev, reps=3, path=CACHE, log=None):
    """Tune the batched form of a Batch and store it under its batch class."""
    import torch
    key = batch_class(b.G, b.m_total)
    mask = torch.empty(max(b.m_total, 1), dtype=torch.uint8, device=b.device)
    sup = torch.empty(max(b.m_total, 1), dtype=torch.int32, device=b.device)
    rounds = torch.empty(max(b.G, 1), dtype=torch.int32, device=b.device)
    best, t, _ = search(b, lambda: kt.ktruss_run_batched(b, K_dev, mask, sup, rounds), None, reps=reps, log=log)
    store(key, best, t, path)
    return key, best, t


if __name__ == "__main__":
    # python -m paper_2009_07929_amd.autotune batch [cache path]: tunes the
    # 4,096-graph batched workload on the GPU and stores its entry.
    import sys
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    if sys.argv[1:2] != ["batch"]:
        raise SystemExit("usage: python -m paper_2009_07929_amd.autotune batch [cache path]")
    path = sys.argv[2] if len(sys.argv) > 2 else CACHE
    p = synth.WORKLOADS["chunglu-batch-4096"].params
    gs = synth.batch_graphs(p["count"], p["seed"], p["nmin"], p["nmax"])
    K = torch.from_numpy(np.array([x[3] for x in gs], np.int32)).cuda()
    b = kt.Batch(kt.build_csrs([(n, s, d) for n, s, d, _ in gs]), device="cuda")
    del gs
    print(tune_batch(b, K, path=path, log=print))
