"""Throughput of the K-truss hot path on one MI355X.

Main workload (default): R-MAT scale 20, edge factor 16 (15.7M edges), K sweep
3, 5, 8, 12.  A step is one full prune-to-fixpoint K-truss run (supports, prune,
repeat until nothing is removed) for every K of the sweep, on a graph already
resident in HBM.  value = edges processed per second = (number of K values x m)
/ step time: the paper's ME/s definition (input edges over the wall time of a
complete K-truss), summed over the sweep.

Extra legs (on by default; --extras picks some, --no-extras skips all), reported
inside the same line:
  batched: 4096 Chung-Lu graphs (K per graph) in one batched run with the
           autotuner's cached schedule and tiles, edges/s = sum of edges /
           batch time, next to the same graphs run one at a time with the plain
           thread-per-edge kernel and with the main schedule.
  learned: R-MAT scale 22 (0.6, 0.2, 0.15, 0.05) and Barabasi-Albert n=4M,
           m=8, K = 3, 6, 10: the learned schedule (trained cost model) next to
           the static degree heuristic, the all-hub schedule and the plain
           kernel, edges/s per K, results checked identical.
  coarse:  the coarse-grained ablation (one thread per row, Algorithm 2's
           granularity) next to the fine-grained thread-per-edge kernel and
           the hub schedule on R-MAT scale 12 (K = 3..6) and scale 20 (K = 3).
  decompose: every edge's trussness on R-MAT scale 20 in one call, next to
           the same levels computed one K at a time from the full graph.

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
SCHEDULES = {"plain": 0, "heuristic": 1, "learned": 2, "wave": 3, "hub": 4, "coarse": 5}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def recorded_traffic(workload, schedule):
    """Per-launch HBM bytes of the support kernel from the rocprofv3 counter runs
    recorded in profiles/traffic.json (FETCH_SIZE and WRITE_SIZE, scaled by the
    copy-kernel calibration); None if none was recorded for this workload and
    schedule, or if the kernel's sources (its file and the shared header)
    changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("%s/%s" % (workload, schedule))
    if not rec:
        return None
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])
    if hashlib.sha256(src).hexdigest() != rec["sources_sha256"]:
        return None
    return (rec["fetch_kib_avg"] * rec["fetch_scale"] + rec["write_kib_avg"] * rec["write_scale"]) * 1024.0


def cpu_baseline(workload, Ks, budget_s=30.0):
    """The CPU oracle (single-threaded C: canonical CSR already built, then the
    level-synchronous peel) timed on a bounded sample of the workload: smaller
    instances of the same R-MAT generator (same a, b, c and edge factor), the
    scale raised one step at a time while the whole K sweep stays within about
    a sixth of `budget_s`.  edges/s = (len(Ks) x sample edges) / sweep time."""
    import oracle
    import synth
    p = synth.WORKLOADS[workload].params
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


def tuning(kt, rounds_per_sync):
    t = kt.ktruss_tuning()
    t.rounds_per_sync = rounds_per_sync
    return t


def first_pass(kt, torch, g, stream, reps=3):
    """Round 1 alone: one support pass over the whole graph (ktruss_support),
    profiled; the hub kernel's time per launch and the pass's merge-model
    bytes (outside the timed region of the step)."""
    sup = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.device)
    kt.ktruss_support(g, None, sup, stream)
    torch.cuda.synchronize()
    kt.ktruss_profile_enable(True)
    for _ in range(reps):
        kt.ktruss_support(g, None, sup, stream)
    torch.cuda.synchronize()
    launches, ms, _, nbytes = kt.ktruss_profile_read(kt.PROFILE_PASS)
    hl, hms, _, _ = kt.ktruss_profile_read(kt.PROFILE_HUB)
    kt.ktruss_profile_enable(False)
    out = {"passes": launches, "pass_ms": ms / max(launches, 1), "bytes": nbytes / max(launches, 1)}
    if hl == launches and hl:
        out["hub_ms"] = hms / hl
        out["achieved_gbps"] = out["bytes"] / (out["hub_ms"] * 1e-3) / 1e9
    return out


def single_sweep(args, kt, torch):
    """The main leg: K sweep on one large graph.  Returns the JSON dict."""
    import synth
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

    g = kt.Graph(rowptr, col, device="cuda:0")
    params = None
    if args.schedule == "learned":
        from paper_2009_07929_amd import cost_model
        params = cost_model.load_params("cuda:0")
        if params is None:
            raise RuntimeError("--schedule learned needs the trained cost-model weights")
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], params, tuning(kt, args.rounds_per_sync))
    mask = torch.empty(m, dtype=torch.uint8, device="cuda:0")
    sup = torch.empty(m, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step():
        for K in Ks:
            kt.ktruss_run(g, K, mask, sup, stream)

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
        per_k[str(K)] = {"rounds": r, "ms": dt * 1e3, "edges_per_s": m / dt, "truss_edges": int(mask.sum().item())}
    # support-pass timing: HIP events on the launch stream, host-loop rounds
    # (graph-replayed rounds are not bracketed by events)
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], params, tuning(kt, 0))
    kt.ktruss_profile_enable(True)
    for K in Ks:
        kt.ktruss_run(g, K, mask, sup, stream)
    torch.cuda.synchronize()
    launches, sup_ms, edge_tasks, nbytes = kt.ktruss_profile_read(kt.PROFILE_PASS)
    kinds = {}
    for name, kind in (("thread", kt.PROFILE_THREAD), ("wave", kt.PROFILE_WAVE), ("hub", kt.PROFILE_HUB),
                       ("hit_sum", kt.PROFILE_HIT_SUM)):
        nl, ms, tasks, _ = kt.ktruss_profile_read(kind)
        if nl:
            kinds[name] = {"launches": nl, "ms": ms, "tasks": tasks}
    kt.ktruss_profile_enable(False)
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], params, tuning(kt, args.rounds_per_sync))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("timed %d steps in %.3fs" % (args.steps, elapsed))

    ms_per_step = elapsed * 1e3 / args.steps
    value = len(Ks) * m * args.steps / elapsed
    avg_pass_ms = sup_ms / max(launches, 1)
    # Dominant kernel: the hub kernel when the schedule launches it (one launch
    # per pass), else the whole pass.  Algorithmic bytes per launch: the merge
    # model of the pass it computes (every task reading its tail and row kappa,
    # three support updates per triangle), as the library's profiler reports.
    bytes_per_launch = nbytes / max(launches, 1)
    hub = kinds.get("hub")
    if hub and hub["launches"] == launches:
        kernel, avg_launch_ms = "k_support_hub", hub["ms"] / hub["launches"]
        traffic = recorded_traffic(args.workload, args.schedule)
    else:
        kernel, avg_launch_ms, traffic = "support pass", avg_pass_ms, None
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if launches else 0.0
    first = first_pass(kt, torch, g, stream)
    del g
    return {
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
                   "rounds_per_sync": args.rounds_per_sync, "per_K": per_k},
        "roofline": {
            "kernel": kernel,
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": traffic,
            "launches": launches,
            "avg_launch_ms": avg_launch_ms,
            "avg_pass_ms": avg_pass_ms,
            "bytes_per_launch": bytes_per_launch,
            "dram_gbps": (traffic / (avg_launch_ms * 1e-3) / 1e9) if traffic else None,
            "variants": kinds,
        },
        "first_pass": first,
    }


def batched_leg(args, kt, torch, count):
    """Batched run of `count` Chung-Lu graphs vs the same graphs one at a time."""
    import numpy as np
    import synth
    t0 = time.perf_counter()
    gs = synth.batch_graphs(count, 5)
    Kg = np.array([g[3] for g in gs], np.int32)
    csr = kt.build_csrs([(n, s, d) for n, s, d, _ in gs])
    del gs
    t_prep = time.perf_counter() - t0
    msum = sum(len(c) for _, c in csr)
    log("batch: %d graphs, %d edges (prep %.1fs)" % (count, msum, t_prep))
    b = kt.Batch(csr, device="cuda:0", schedule=SCHEDULES[args.schedule])
    b.c.tuning = tuning(kt, args.rounds_per_sync)
    cfg = None
    if not args.no_autotune:  # the autotuner's cached choice for this batch class, if any
        from paper_2009_07929_amd import autotune
        key = autotune.batch_class(b.G, b.m_total)
        if key in autotune.load_cache():
            cfg = autotune.tuned_config(key)
            autotune.apply(b, cfg)
    K_d = torch.from_numpy(Kg).cuda()
    mask = torch.empty(b.m_total, dtype=torch.uint8, device="cuda:0")
    sup = torch.empty(b.m_total, dtype=torch.int32, device="cuda:0")
    rounds = torch.empty(b.G, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    kt.ktruss_run_batched(b, K_d, mask, sup, rounds, stream)      # warm-up
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        kt.ktruss_run_batched(b, K_d, mask, sup, rounds, stream)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    batch_rounds = rounds.cpu().numpy()
    out = {"workload": "chunglu-batch-%d" % count, "graphs": count, "edges": msum,
           "batched_edges_per_s": msum / t_batch, "batched_ms": t_batch * 1e3,
           "max_rounds": int(batch_rounds.max()),
           "schedule": cfg["schedule"] if cfg else args.schedule, "autotuned": cfg}
    del b, mask, sup
    if args.no_per_graph:
        return out
    # the same graphs one at a time (graph and output buffers resident before timing)
    for name in ("plain", args.schedule):
        graphs = [kt.Graph(rp, c, device="cuda:0", schedule=SCHEDULES[name]) for rp, c in csr]
        outs = [(torch.empty(max(len(c), 1), dtype=torch.uint8, device="cuda:0"),
                 torch.empty(max(len(c), 1), dtype=torch.int32, device="cuda:0")) for _, c in csr]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        agree = True
        for i, g in enumerate(graphs):
            _, _, r = kt.ktruss_run(g, int(Kg[i]), outs[i][0], outs[i][1], stream)
            agree &= r == int(batch_rounds[i])
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        out["per_graph_%s_edges_per_s" % name] = msum / t_seq
        out["per_graph_%s_ms" % name] = t_seq * 1e3
        out["rounds_agree_%s" % name] = bool(agree)
        del graphs, outs
    out["batched_vs_plain"] = out["batched_edges_per_s"] / out["per_graph_plain_edges_per_s"]
    return out


def learned_leg(args, kt, torch, workloads=("rmat-s22-ef16", "ba-4M-m8")):
    """The learned schedule (trained cost model) against the static degree
    heuristic, the all-hub schedule and the plain thread-per-edge kernel on
    the evaluation graphs: edges/s per K (median of three runs unless one run
    takes over a second), results checked equal across schedules."""
    import numpy as np
    import synth
    from paper_2009_07929_amd import cost_model
    params = cost_model.load_params("cuda:0")
    if params is None:
        return {"error": "no trained cost-model weights"}
    out = {}
    stream = torch.cuda.current_stream()
    for wname in workloads:
        w = synth.WORKLOADS[wname]
        n, s, d = synth.workload_pairs(wname)
        rowptr, col, _ = kt.ktruss_build_csr(s, d, n)
        del s, d
        m = len(col)
        g = kt.Graph(rowptr, col, device="cuda:0")
        mask = torch.empty(m, dtype=torch.uint8, device="cuda:0")
        sup = torch.empty(m, dtype=torch.int32, device="cuda:0")
        res = {"n": n, "m": m}
        digest = {}
        for sname in ("plain", "heuristic", "learned", "hub"):
            kt.ktruss_set_schedule(g, SCHEDULES[sname], params if sname == "learned" else None, tuning(kt, 0))
            per = {}
            for K in w.Ks:
                kt.ktruss_run(g, K, mask, sup, stream)  # warm-up
                ts = []
                while not ts or (len(ts) < 3 and ts[0] < 1.0):  # median of 3 unless a run takes seconds
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, _, r = kt.ktruss_run(g, K, mask, sup, stream)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                dt = float(np.median(ts))
                dg = (r, int(mask.sum().item()), int(sup.to(torch.int64).sum().item()))
                if digest.setdefault(K, dg) != dg:
                    raise RuntimeError("schedule %s disagrees on %s K=%d" % (sname, wname, K))
                per[str(K)] = {"ms": dt * 1e3, "edges_per_s": m / dt, "rounds": r}
            tot = sum(v["ms"] for v in per.values())
            res[sname] = {"per_K": per, "edges_per_s": len(w.Ks) * m / (tot * 1e-3)}
            log("learned leg: %s %s %.3e edges/s" % (wname, sname, res[sname]["edges_per_s"]))
        res["learned_vs_heuristic"] = res["learned"]["edges_per_s"] / res["heuristic"]["edges_per_s"]
        res["learned_vs_plain"] = res["learned"]["edges_per_s"] / res["plain"]["edges_per_s"]
        res["learned_vs_hub"] = res["learned"]["edges_per_s"] / res["hub"]["edges_per_s"]
        out[wname] = res
        del g, mask, sup
    return out


def coarse_leg(args, kt, torch, workloads=(("rmat-s12-ef8", None), ("rmat-s20-ef16", (3,)))):
    """The coarse-grained ablation: one thread per row running its edge tasks
    in turn (Algorithm 2's granularity) against the fine-grained thread-per-
    edge kernel and the hub schedule, edges/s per K (median of three runs
    unless one run takes over a second), results checked equal."""
    import numpy as np
    import synth
    out = {}
    stream = torch.cuda.current_stream()
    for wname, Ks in workloads:
        w = synth.WORKLOADS[wname]
        Ks = Ks or w.Ks
        n, s, d = synth.workload_pairs(wname)
        rowptr, col, _ = kt.ktruss_build_csr(s, d, n)
        del s, d
        m = len(col)
        g = kt.Graph(rowptr, col, device="cuda:0")
        mask = torch.empty(max(m, 1), dtype=torch.uint8, device="cuda:0")
        sup = torch.empty(max(m, 1), dtype=torch.int32, device="cuda:0")
        res = {"n": n, "m": m, "Ks": list(Ks)}
        digest = {}
        for sname in ("coarse", "plain", "hub"):
            kt.ktruss_set_schedule(g, SCHEDULES[sname], None, tuning(kt, 0))
            per = {}
            for K in Ks:
                kt.ktruss_run(g, K, mask, sup, stream)  # warm-up
                ts = []
                while not ts or (len(ts) < 3 and ts[0] < 1.0):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, _, r = kt.ktruss_run(g, K, mask, sup, stream)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                dt = float(np.median(ts))
                dg = (r, int(mask[:m].sum().item()), int(sup[:m].to(torch.int64).sum().item()))
                if digest.setdefault(K, dg) != dg:
                    raise RuntimeError("schedule %s disagrees on %s K=%d" % (sname, wname, K))
                per[str(K)] = {"ms": dt * 1e3, "edges_per_s": m / dt, "rounds": r}
            tot = sum(v["ms"] for v in per.values())
            res[sname] = {"per_K": per, "edges_per_s": len(Ks) * m / (tot * 1e-3)}
            log("coarse leg: %s %s %.3e edges/s" % (wname, sname, res[sname]["edges_per_s"]))
        res["fine_vs_coarse"] = res["plain"]["edges_per_s"] / res["coarse"]["edges_per_s"]
        res["hub_vs_coarse"] = res["hub"]["edges_per_s"] / res["coarse"]["edges_per_s"]
        out[wname] = res
        del g, mask, sup
    return out


def decompose_leg(args, kt, torch, wname="rmat-s20-ef16"):
    """Truss decomposition (every edge's trussness, K_max) in one call, next
    to the same trusses computed one K at a time from the full graph
    (ktruss_run for K = 3 .. K_max + 1); the trussness is checked against
    those runs."""
    import numpy as np
    import synth
    n, s, d = synth.workload_pairs(wname)
    rowptr, col, _ = kt.ktruss_build_csr(s, d, n)
    del s, d
    m = len(col)
    g = kt.Graph(rowptr, col, device="cuda:0")
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], None, tuning(kt, 0))
    stream = torch.cuda.current_stream()
    tr = torch.empty(m, dtype=torch.int32, device="cuda:0")
    kt.ktruss_decompose(g, tr, stream)  # warm-up
    ts = []
    while not ts or (len(ts) < 3 and ts[0] < 1.0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, k_max = kt.ktruss_decompose(g, tr, stream)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_dec = float(np.median(ts))
    # the same levels one K at a time, each from the full graph
    mask = torch.empty(m, dtype=torch.uint8, device="cuda:0")
    sup = torch.empty(m, dtype=torch.int32, device="cuda:0")
    level = torch.full((m,), 2, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for K in range(3, k_max + 2):
        kt.ktruss_run(g, K, mask, sup, stream)
        level[mask.bool()] = K
    torch.cuda.synchronize()
    t_each = time.perf_counter() - t0
    agree = bool(torch.equal(level, tr))
    if not agree:
        raise RuntimeError("decomposition disagrees with the per-K runs on %s" % wname)
    del g
    return {"workload": wname, "m": m, "k_max": k_max, "decompose_ms": t_dec * 1e3, "edges_per_s": m / t_dec,
            "per_K_runs_ms": t_each * 1e3, "speedup_vs_per_K_runs": t_each / t_dec, "agree": agree}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat-s20-ef16")
    ap.add_argument("--ks", default=None, help="comma-separated K values (default: the workload's)")
    ap.add_argument("--schedule", default="hub", choices=sorted(SCHEDULES))
    ap.add_argument("--rounds-per-sync", type=int, default=0,
                    help="prune rounds replayed from a hipGraph per host check (<= 1: host loop)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="batched,learned,coarse,decompose",
                    help="comma-separated extra legs to run after the main leg (batched, learned, coarse, decompose)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched leg: ignore the autotuner's cached configuration")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--no-per-graph", action="store_true",
                    help="batched leg without the one-graph-at-a-time baselines (for profiling the batched run)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed region, copy a device buffer of this size 3 times (a plain copy "
                         "kernel of known traffic, for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each GPU would run its own graphs; see the sharding notes in the design document).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_07929_amd import ktruss as kt

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    out = single_sweep(args, kt, torch)

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    extras = set() if args.no_extras else {e for e in args.extras.split(",") if e}
    unknown = extras - {"batched", "learned", "coarse", "decompose"}
    if unknown:
        raise SystemExit("unknown extra legs: %s" % ",".join(sorted(unknown)))
    if "batched" in extras:
        log("batched leg ...")
        out["batched"] = batched_leg(args, kt, torch, args.batch_graphs)
    if "learned" in extras:
        log("learned-schedule leg ...")
        out["learned"] = learned_leg(args, kt, torch)
    if "coarse" in extras:
        log("coarse-grained ablation leg ...")
        out["coarse"] = coarse_leg(args, kt, torch)
    if "decompose" in extras:
        log("truss decomposition leg ...")
        out["decompose"] = decompose_leg(args, kt, torch)
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.workload, tuple(out["config"]["Ks"]), args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
