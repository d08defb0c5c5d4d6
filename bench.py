"""Throughput of the K-truss hot path on one MI355X.

A step is one full prune-to-fixpoint K-truss run (supports, prune, repeat until
nothing is removed) for every K of the workload's K sweep, on a graph already
resident in HBM.  value = edges processed per second = (number of K values x m)
/ step time, the paper's ME/s definition (input edges over wall time of a
complete K-truss), summed over the sweep.

Prints one JSON line (rank 0).  Only one GPU is used; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(workload, Ks, budget_s=30.0):
    """The CPU oracle (single-threaded C: canonical CSR already built, then the
    level-synchronous peel) timed on a bounded sample of the workload: smaller
    instances of the same R-MAT generator (same a, b, c and edge factor), the
    scale raised one step at a time while the whole K sweep stays within about
    a third of `budget_s`.  edges/s = (len(Ks) x sample edges) / sweep time."""
    import oracle
    import synth
    w = synth.WORKLOADS[workload]
    p = w.params
    if "scale" not in p:
        return None
    a, b, c = p["abc"]
    last = None
    for scale in range(12, p["scale"] + 1):
        n, s, d = synth.rmat(scale, p["edge_factor"], a, b, c, p["seed"])
        rp, col, _ = oracle.canonical_csr(n, s, d)
        t0 = time.perf_counter()
        for K in Ks:
            oracle.truss(rp, col, K, "P")
        dt = time.perf_counter() - t0
        last = (scale, len(col), dt)
        if dt > budget_s / 6:
            break
    scale, msub, dt = last
    return {"value": len(Ks) * msub / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "oracle mode P, one thread, K sweep %s on R-MAT scale %d (same a,b,c, edge factor %d, "
                      "seed %d): m=%d, %.2f s" % (list(Ks), scale, p["edge_factor"], p["seed"], msub, dt)}


def recorded_traffic(workload, schedule):
    """Per-launch HBM bytes of the support kernel from the rocprofv3 counter runs
    recorded in profiles/traffic.json (FETCH_SIZE and WRITE_SIZE, scaled by the
    copy-kernel calibration); None if none was recorded for this workload and
    schedule, or if the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("%s/%s" % (workload, schedule))
    if not rec:
        return None
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return (rec["fetch_kib_avg"] * rec["fetch_scale"] + rec["write_kib_avg"] * rec["write_scale"]) * 1024.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat-s20-ef16")
    ap.add_argument("--ks", default=None, help="comma-separated K values (default: the workload's)")
    ap.add_argument("--schedule", default="hub", choices=["plain", "heuristic", "learned", "wave", "hub"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed region, copy a device buffer of this size 3 times (a plain copy "
                         "kernel of known traffic, for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each GPU would run its own graphs; see the sharding notes in the design document).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2009_07929_amd import ktruss as kt

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.WORKLOADS[args.workload]
    Ks = tuple(int(k) for k in args.ks.split(",")) if args.ks else w.Ks
    t0 = time.perf_counter()
    n, s, d = synth.workload_pairs(args.workload)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    rowptr, col, _ = kt.ktruss_build_csr(s, d, n)
    t_build = time.perf_counter() - t0
    del s, d
    m = len(col)
    log("workload %s: n=%d m=%d (gen %.1fs, csr %.1fs)" % (args.workload, n, m, t_gen, t_build))

    sched = {"plain": kt.SCHED_PLAIN, "heuristic": kt.SCHED_HEURISTIC, "learned": kt.SCHED_LEARNED,
             "wave": kt.SCHED_FORCE_WAVE, "hub": kt.SCHED_FORCE_HUB}[args.schedule]
    g = kt.Graph(rowptr, col, device="cuda:0")
    kt.ktruss_set_schedule(g, sched)
    mask = torch.empty(m, dtype=torch.uint8, device="cuda:0")
    sup = torch.empty(m, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step():
        rounds = []
        for K in Ks:
            _, _, r = kt.ktruss_run(g, K, mask, sup, stream)
            rounds.append(r)
        return rounds

    for i in range(args.warmup):
        step()
        log("warmup %d done" % i)
    # per-K wall time and rounds (one untimed pass, outside the timed region)
    per_k = {}
    for K in Ks:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, r = kt.ktruss_run(g, K, mask, sup, stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per_k[str(K)] = {"rounds": r, "ms": dt * 1e3, "edges_per_s": m / dt,
                         "truss_edges": int(mask.sum().item())}
    kt.ktruss_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, sup_ms, edge_tasks, nbytes = kt.ktruss_profile_read(kt.PROFILE_PASS)
    kinds = {}
    for name, kind in (("thread", kt.PROFILE_THREAD), ("wave", kt.PROFILE_WAVE), ("hub", kt.PROFILE_HUB)):
        nl, ms, tasks, _ = kt.ktruss_profile_read(kind)
        if nl:
            kinds[name] = {"launches": nl, "ms": ms, "tasks": tasks}
    kt.ktruss_profile_enable(False)
    log("timed %d steps in %.3fs" % (args.steps, elapsed))

    ms_per_step = elapsed * 1e3 / args.steps
    value = len(Ks) * m * args.steps / elapsed
    avg_launch_ms = sup_ms / max(launches, 1)
    achieved = (nbytes / max(launches, 1)) / (avg_launch_ms * 1e-3) / 1e9 if launches else 0.0

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.workload, Ks, args.cpu_budget)

    out = {
        "metric": "edges processed/s per K + HBM GB/s; learned/batched vs plain GPU, bit-exact",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "Ks": list(Ks), "schedule": args.schedule,
                   "per_K": per_k},
        "roofline": {
            "kernel": "support pass",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": recorded_traffic(args.workload, args.schedule),
            "launches": launches,
            "avg_launch_ms": avg_launch_ms,
            "support_share_of_step": sup_ms / (elapsed * 1e3),
            "variants": kinds,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
