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
    schedule (which name the run: e.g. "rmat-s23-ef16-clique600/hub/inc2"), or
    if the kernel's sources (its file and the shared header) changed since."""
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


def cpu_baseline(workload, Ks, budget_s=20.0, seed=7):
    """The CPU oracle (single-threaded C, pinned to one core) timed on a bounded
    sample of the bench graph itself: the oracle's own canonical CSR of the
    workload, then its support evaluation (triangles containing the edge,
    Algorithm 1's S = (A^T A) o A read at one edge) of uniformly sampled edge
    positions, the sample doubled until the loop takes budget_s / 4 or more.
    Every K of a sweep needs at least one full support evaluation of the whole
    graph, so edges/s = sample edges / loop seconds bounds the oracle's sweep
    rate (K values x m / sweep time) from above."""
    import numpy as np
    import oracle
    import synth
    host_cpus = os.cpu_count()
    pinned = None
    if hasattr(os, "sched_setaffinity"):
        before = os.sched_getaffinity(0)
        pinned = min(before)
        os.sched_setaffinity(0, {pinned})
    try:
        n, s, d = synth.workload_pairs(workload)
        t0 = time.perf_counter()
        rp, col, _ = oracle.canonical_csr(n, s, d)
        t_csr = time.perf_counter() - t0
        del s, d
        m = len(col)
        rng = np.random.default_rng(seed)
        k = 1024
        while True:
            edges = np.sort(rng.choice(m, size=min(k, m), replace=False)).astype(np.int64)
            _, dt = oracle.supports_of(rp, col, edges, timed=True)
            if dt >= budget_s / 4 or k >= m:
                break
            k *= 2
    finally:
        if pinned is not None:
            os.sched_setaffinity(0, before)
    return {"value": len(edges) / dt, "unit": "edges/s", "cores": 1, "host_cpus": host_cpus, "kind": "oracle",
            "pinned_cpu": pinned,
            "sample": "oracle support evaluation of %d uniformly sampled edges of %s (m=%d; oracle canonical CSR "
                      "built in %.1f s, not timed), one thread pinned to one core, %.2f s; an upper bound of the "
                      "oracle's rate on the K sweep %s, each K of which needs a whole support evaluation"
                      % (len(edges), workload, m, t_csr, dt, list(Ks))}


def tuning(kt, rounds_per_sync, incremental=0, peel_ratio=0):
    t = kt.ktruss_tuning()
    t.rounds_per_sync = rounds_per_sync
    t.incremental = incremental
    t.peel_ratio = peel_ratio
    return t


def hub_model_bytes(st):
    """Algorithmic bytes of the workgroup-per-hub-row kernel over the profiled
    passes (Algorithm 3's tasks, grouped by row kappa): every hub task reads
    its tail once (4 B per element) and its descriptor (edge, row and tail
    length, 12 B), adds into S(i, kappa) (8 B read-modify-write) and writes
    its hit words (8 B each); every staged row-kappa element is read once
    (4 B) and its support S(kappa, w) read and written once (8 B)."""
    return (4 * st["hub_tail"] + 20 * st["hub_tasks"] + 8 * st["hub_words"] + 12 * st["hub_staged"])


def merge_model_bytes(st):
    """The merge model of a support pass: every task reads its row-i tail and
    row kappa (4 B per element) and col[e], rowptr[kappa], rowptr[kappa+1],
    and three support atomics per triangle plus one per task (8 B each)."""
    T = st["support"] // 3
    return 4 * (3 * st["edges"] + st["tail"] + st["rowk"]) + 8 * (2 * T + st["edges"])


def first_pass(kt, torch, g, stream, workload, schedule, reps=3):
    """Round 1 alone: one support pass over the whole graph (ktruss_support),
    profiled; the hub kernel's time per launch and the pass's algorithmic
    bytes (outside the timed region of the step)."""
    sup = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.device)
    kt.ktruss_support(g, None, sup, stream)
    torch.cuda.synchronize()
    kt.ktruss_profile_enable(True)
    for _ in range(reps):
        kt.ktruss_support(g, None, sup, stream)
    torch.cuda.synchronize()
    launches, ms, _, _ = kt.ktruss_profile_read(kt.PROFILE_PASS)
    hl, hms, _, _ = kt.ktruss_profile_read(kt.PROFILE_HUB)
    st = kt.ktruss_profile_stats()
    kt.ktruss_profile_enable(False)
    out = {"passes": launches, "pass_ms": ms / max(launches, 1),
           "algorithmic_bytes": hub_model_bytes(st) / max(launches, 1),
           "merge_model_bytes": merge_model_bytes(st) / max(launches, 1)}
    if hl == launches and hl:
        out["hub_ms"] = hms / hl
        out["achieved_gbps"] = out["algorithmic_bytes"] / (out["hub_ms"] * 1e-3) / 1e9
        out["merge_model_gbps"] = out["merge_model_bytes"] / (out["hub_ms"] * 1e-3) / 1e9
        traffic = recorded_traffic(workload + "/round1", schedule)
        out["traffic"] = traffic
        out["dram_gbps"] = traffic / (out["hub_ms"] * 1e-3) / 1e9 if traffic else None
    return out


def sweep(args, kt, torch, workload, Ks, steps, warmup, rounds_per_sync):
    """A K sweep on one large graph resident in HBM: per-K rounds and times,
    the support launches profiled by kind with their pass statistics, then
    `steps` timed sweeps.  Returns the fields of the bench line."""
    import synth
    t0 = time.perf_counter()
    n, s, d = synth.workload_pairs(workload)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    rowptr, col, _ = kt.ktruss_build_csr(s, d, n)
    t_build = time.perf_counter() - t0
    del s, d
    m = len(col)
    log("workload %s: n=%d m=%d (gen %.1fs, csr %.1fs)" % (workload, n, m, t_gen, t_build))

    g = kt.Graph(rowptr, col, device="cuda:0")
    params = None
    if args.schedule == "learned":
        from paper_2009_07929_amd import cost_model
        params = cost_model.load_params("cuda:0")
        if params is None:
            raise RuntimeError("--schedule learned needs the trained cost-model weights")
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], params,
                           tuning(kt, rounds_per_sync, args.incremental, args.peel_ratio))
    mask = torch.empty(m, dtype=torch.uint8, device="cuda:0")
    sup = torch.empty(m, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()

    def step():
        for K in Ks:
            kt.ktruss_run(g, K, mask, sup, stream)

    for i in range(warmup):
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
        log("K=%d: %d rounds, %.1f ms" % (K, r, dt * 1e3))
    # support-pass timing: HIP events on the launch stream, host-loop rounds
    # (graph-replayed rounds are not bracketed by events)
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], params, tuning(kt, 0, args.incremental, args.peel_ratio))
    kt.ktruss_profile_enable(True)
    for K in Ks:
        kt.ktruss_run(g, K, mask, sup, stream)
    torch.cuda.synchronize()
    launches, sup_ms, _, _ = kt.ktruss_profile_read(kt.PROFILE_PASS)
    kinds = {}
    for name, kind in (("thread", kt.PROFILE_THREAD), ("wave", kt.PROFILE_WAVE), ("hub", kt.PROFILE_HUB),
                       ("hit_sum", kt.PROFILE_HIT_SUM), ("row", kt.PROFILE_ROW)):
        nl, ms, tasks, _ = kt.ktruss_profile_read(kind)
        if nl:
            kinds[name] = {"launches": nl, "ms": ms, "tasks": tasks}
    st = kt.ktruss_profile_stats()
    kt.ktruss_profile_enable(False)
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], params,
                           tuning(kt, rounds_per_sync, args.incremental, args.peel_ratio))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("timed %d steps in %.3fs" % (steps, elapsed))

    ms_per_step = elapsed * 1e3 / max(steps, 1)
    avg_pass_ms = sup_ms / max(launches, 1)
    # Dominant kernel: the hub kernel when the schedule launches it once per
    # pass; its algorithmic bytes per launch follow the hub model, the merge
    # model's bytes (what a plain per-task merge would read) are reported
    # beside them.
    hub = kinds.get("hub")
    hub_bytes, mm_bytes = hub_model_bytes(st), merge_model_bytes(st)
    if hub and hub["launches"] == launches:
        kernel, avg_launch_ms = "k_support_hub", hub["ms"] / hub["launches"]
        bytes_per_launch = hub_bytes / launches
        traffic = recorded_traffic(workload, "%s/inc%d" % (args.schedule, args.incremental))
    else:
        kernel, avg_launch_ms, traffic = "support pass", avg_pass_ms, None
        bytes_per_launch = mm_bytes / max(launches, 1)
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if launches else 0.0
    roofline = {
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
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "dram_gbps": (traffic / (avg_launch_ms * 1e-3) / 1e9) if traffic else None,
        "dram_frac": (traffic / (avg_launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS) if traffic else None,
        "merge_model_bytes_per_launch": mm_bytes / max(launches, 1),
        "cache_leverage": (mm_bytes / max(launches, 1) / traffic) if traffic else None,
        "sweep_algorithmic_gbps": (hub_bytes if kernel == "k_support_hub" else mm_bytes)
                                  / max(sum(v["ms"] for v in per_k.values()), 1e-9) / 1e6,
        "pass_stats": st,
        "variants": kinds,
    }
    first = first_pass(kt, torch, g, stream, workload, args.schedule)
    del g
    return {"n": n, "m": m, "Ks": list(Ks), "per_K": per_k, "steps": steps, "ms_per_step": ms_per_step,
            "value": len(Ks) * m * steps / elapsed if steps else 0.0, "roofline": roofline, "first_pass": first}


def main_line(args, kt, torch):
    """The main leg: the K sweep of the bench workload.  Returns the JSON dict."""
    import synth
    w = synth.WORKLOADS[args.workload]
    Ks = tuple(int(k) for k in args.ks.split(",")) if args.ks else w.Ks
    r = sweep(args, kt, torch, args.workload, Ks, args.steps, args.warmup, args.rounds_per_sync)
    return {
        "metric": "edges processed/s per K + HBM GB/s; learned/batched vs plain GPU, bit-exact",
        "value": r["value"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": r["n"], "m": r["m"], "Ks": r["Ks"], "schedule": args.schedule,
                   "rounds_per_sync": args.rounds_per_sync, "incremental": args.incremental,
                   "peel_ratio": args.peel_ratio, "per_K": r["per_K"]},
        "roofline": r["roofline"],
        "first_pass": r["first_pass"],
    }


def s20_leg(args, kt, torch, workload="rmat-s20-ef16"):
    """The scale-20 R-MAT sweep (K = 3, 5, 8, 12) under the bench schedule."""
    import synth
    r = sweep(args, kt, torch, workload, synth.WORKLOADS[workload].Ks, 5, 1, args.rounds_per_sync)
    r["workload"] = workload
    r["edges_per_s"] = r.pop("value")
    return r


def batched_leg(args, kt, torch, count):
    """Batched run of `count` Chung-Lu graphs (the autotuned schedule, then the
    plain thread-per-edge kernel in the same one batched call) vs the same
    graphs one at a time; every per-graph run is compared element by element
    with the batched masks and supports."""
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
    if cfg is None:
        b.c.tuning.incremental = args.incremental
        b.c.tuning.peel_ratio = args.peel_ratio
    K_d = torch.from_numpy(Kg).cuda()
    mask = torch.empty(b.m_total, dtype=torch.uint8, device="cuda:0")
    sup = torch.empty(b.m_total, dtype=torch.int32, device="cuda:0")
    rounds = torch.empty(b.G, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()

    def timed_batch(reps=3):
        kt.ktruss_run_batched(b, K_d, mask, sup, rounds, stream)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            kt.ktruss_run_batched(b, K_d, mask, sup, rounds, stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_batch = timed_batch()
    batch_rounds = rounds.cpu().numpy()
    out = {"workload": "chunglu-batch-%d" % count, "graphs": count, "edges": msum,
           "batched_edges_per_s": msum / t_batch, "batched_ms": t_batch * 1e3,
           "max_rounds": int(batch_rounds.max()),
           "schedule": cfg["schedule"] if cfg else args.schedule, "autotuned": cfg,
           "incremental": int(b.c.tuning.incremental), "peel_ratio": float(b.c.tuning.peel_ratio)}
    if args.no_per_graph:
        del b, mask, sup
        return out
    # the plain thread-per-edge kernel on the same union in one batched call
    mask_ref, sup_ref = mask.clone(), sup.clone()
    b.c.schedule = SCHEDULES["plain"]
    t_plain_batch = timed_batch()
    if not (torch.equal(mask, mask_ref) and torch.equal(sup, sup_ref)
            and np.array_equal(rounds.cpu().numpy(), batch_rounds)):
        raise RuntimeError("batched run under the plain kernel disagrees with the autotuned schedule")
    out["batched_plain_edges_per_s"] = msum / t_plain_batch
    out["batched_plain_ms"] = t_plain_batch * 1e3
    del b, mask, sup
    eo = np.concatenate([[0], np.cumsum([len(c) for _, c in csr])]).astype(np.int64)
    # the same graphs one at a time (graph and output buffers resident before timing)
    for name in ("plain", args.schedule):
        graphs = [kt.Graph(rp, c, device="cuda:0", schedule=SCHEDULES[name]) for rp, c in csr]
        outs = [(torch.empty(max(len(c), 1), dtype=torch.uint8, device="cuda:0"),
                 torch.empty(max(len(c), 1), dtype=torch.int32, device="cuda:0")) for _, c in csr]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = []
        for i, g in enumerate(graphs):
            _, _, r = kt.ktruss_run(g, int(Kg[i]), outs[i][0], outs[i][1], stream)
            rs.append(r)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        for i in range(count):  # element by element against the batched run
            mi = len(csr[i][1])
            if rs[i] != int(batch_rounds[i]) or not (
                    torch.equal(outs[i][0][:mi], mask_ref[eo[i]:eo[i + 1]])
                    and torch.equal(outs[i][1][:mi], sup_ref[eo[i]:eo[i + 1]])):
                raise RuntimeError("graph %d: per-graph %s run disagrees with the batched run" % (i, name))
        out["per_graph_%s_edges_per_s" % name] = msum / t_seq
        out["per_graph_%s_ms" % name] = t_seq * 1e3
        out["agree_%s" % name] = True
        del graphs, outs
    out["batched_vs_plain"] = out["batched_edges_per_s"] / out["per_graph_plain_edges_per_s"]
    out["batched_vs_batched_plain"] = out["batched_edges_per_s"] / out["batched_plain_edges_per_s"]
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


def incremental_leg(args, kt, torch, cases=(("rmat-s20-ef16", (5, 8, 12)),
                                           ("rmat-s23-ef16-clique600", (3, 10, 50, 600)))):
    """Incremental support maintenance (the survivors keep their supports and
    each prune takes off the triangles it destroys) against recomputing every
    pass (Algorithm 1), under the bench schedule: per K the time of a whole
    run (median of three unless a run takes over a second) in both modes and
    in the auto mode, results checked identical."""
    import numpy as np
    import synth
    out = {}
    stream = torch.cuda.current_stream()
    for wname, Ks in cases:
        n, s, d = synth.workload_pairs(wname)
        rowptr, col, _ = kt.ktruss_build_csr(s, d, n)
        del s, d
        m = len(col)
        g = kt.Graph(rowptr, col, device="cuda:0")
        mask = torch.empty(m, dtype=torch.uint8, device="cuda:0")
        sup = torch.empty(m, dtype=torch.int32, device="cuda:0")
        res = {"n": n, "m": m, "Ks": list(Ks), "schedule": args.schedule}
        ref = {}
        for mode, ratio, label in ((0, 0, "recompute"), (1, 0, "incremental"), (2, args.peel_ratio, "auto")):
            kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], None, tuning(kt, 0, mode, ratio))
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
                if K not in ref:
                    ref[K] = (r, mask.clone(), sup.clone())
                elif not (r == ref[K][0] and torch.equal(mask, ref[K][1]) and torch.equal(sup, ref[K][2])):
                    raise RuntimeError("%s mode disagrees with recompute on %s K=%d" % (label, wname, K))
                dt = float(np.median(ts))
                per[str(K)] = {"ms": dt * 1e3, "edges_per_s": m / dt, "rounds": r}
            tot = sum(v["ms"] for v in per.values())
            res[label] = {"per_K": per, "edges_per_s": len(Ks) * m / (tot * 1e-3)}
            log("incremental leg: %s %s %.3e edges/s" % (wname, label, res[label]["edges_per_s"]))
        res["incremental_vs_recompute"] = res["incremental"]["edges_per_s"] / res["recompute"]["edges_per_s"]
        res["auto_vs_recompute"] = res["auto"]["edges_per_s"] / res["recompute"]["edges_per_s"]
        out[wname] = res
        del g, mask, sup, ref
    return out


def butterfly_leg(args, kt, torch, wname="bip-cl-1M-16M"):
    """Butterfly counting (per edge and total) on a power-law bipartite graph:
    time of one ktruss_butterflies call (median of three), edges/s, and the
    invariant that every butterfly has four edges (sum of per-edge counts =
    4 x total)."""
    import numpy as np
    import synth
    nu, nv, u, v = synth.bipartite_pairs(wname)
    rp, col = synth.bipartite_csr(nu, nv, u, v)
    del u, v
    m = len(col)
    rp_d = torch.from_numpy(rp).cuda()
    col_d = torch.from_numpy(col).cuda()
    count = torch.empty(m, dtype=torch.int64, device="cuda:0")
    work = torch.empty(kt.ktruss_butterfly_workspace_bytes(nu, nv, m) + 256, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream()
    kt.ktruss_butterflies(nu, nv, rp_d, col_d, count=count, stream=stream, work=work)  # warm-up
    ts = []
    while not ts or (len(ts) < 3 and ts[0] < 1.0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, total = kt.ktruss_butterflies(nu, nv, rp_d, col_d, count=count, stream=stream, work=work)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    csum = int(count.sum().item())
    if csum != 4 * total:
        raise RuntimeError("butterfly counts: sum of edge counts %d != 4 x total %d" % (csum, total))
    du = np.diff(rp).astype(np.int64)
    dv = np.bincount(col, minlength=nv).astype(np.int64)
    return {"workload": wname, "nu": nu, "nv": nv, "m": m, "butterflies": total, "ms": dt * 1e3,
            "edges_per_s": m / dt, "wedges_centred_u": int((du * (du - 1) // 2).sum()),
            "wedges_centred_v": int((dv * (dv - 1) // 2).sum()), "sum_of_edge_counts_is_4x_total": True}


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
    kt.ktruss_set_schedule(g, SCHEDULES[args.schedule], None,
                           tuning(kt, 0, args.incremental, args.peel_ratio))
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
            "per_K_runs_ms": t_each * 1e3, "speedup_vs_per_K_runs": t_each / t_dec, "agree": agree,
            "incremental": args.incremental}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat-s23-ef16-clique600")
    ap.add_argument("--ks", default=None, help="comma-separated K values (default: the workload's)")
    ap.add_argument("--schedule", default="hub", choices=sorted(SCHEDULES))
    ap.add_argument("--incremental", type=int, default=2, choices=(0, 1, 2),
                    help="support maintenance of the main legs: 0 recompute every pass, 1 peel after every prune, "
                         "2 peel unless a prune removes more than --peel-ratio x the survivors")
    ap.add_argument("--peel-ratio", type=float, default=0.0,
                    help="incremental 2: peel unless a prune removes more than this x the survivors (0: the "
                         "library default, 0.125)")
    ap.add_argument("--rounds-per-sync", type=int, default=0,
                    help="prune rounds replayed from a hipGraph per host check (<= 1: host loop)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="s20,incremental,batched,learned,coarse,decompose,butterfly",
                    help="comma-separated extra legs to run after the main leg (s20, incremental, batched, "
                         "learned, coarse, decompose, butterfly)")
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
    out = main_line(args, kt, torch)

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    extras = set() if args.no_extras else {e for e in args.extras.split(",") if e}
    unknown = extras - {"s20", "incremental", "batched", "learned", "coarse", "decompose", "butterfly"}
    if unknown:
        raise SystemExit("unknown extra legs: %s" % ",".join(sorted(unknown)))
    if "s20" in extras:
        log("R-MAT scale 20 leg ...")
        out["s20"] = s20_leg(args, kt, torch)
    if "incremental" in extras:
        log("incremental maintenance leg ...")
        out["incremental"] = incremental_leg(args, kt, torch)
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
    if "butterfly" in extras:
        log("butterfly leg ...")
        out["butterfly"] = butterfly_leg(args, kt, torch)
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.workload, tuple(out["config"]["Ks"]), args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
