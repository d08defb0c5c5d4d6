"""Writes tests/golden/digests.json: the oracle's K-truss results on the full-size
synthetic workloads, reduced to digests so that the GPU tests can compare bit
for bit without storing per-edge arrays.

Uses only the input generators (synth) and the CPU oracle (oracle/, mode P,
its own canonicalisation).  Every K runs from the full graph, exactly as
ktruss_run does, so the pass counts are comparable.  For each (workload, K):
  m, n, rounds, truss_edges, support_sum,
  mask_sha256     sha256 of the uint8 mask in canonical edge order,
  support_sha256  sha256 of the little-endian int32 supports in canonical order,
  keyed_sha256    sha256 of the survivors as little-endian int64 triples
                  (min original id, max original id, support), sorted.
The keyed digest does not depend on the relabelling, so a builder bug cannot
hide behind it.

The batched workload (chunglu-batch-4096: every graph with its own K) is
stored per graph as pass counts, truss sizes and support sums, plus one
sha256 over the graphs' mask digests and one over their support digests, in
graph order (each graph's digest as above, in its own canonical edge order).

Runs:
  python tests/golden/make_digests.py [workload ...]
      sequentially, straight into digests.json (default: the two small ones);
  python tests/golden/make_digests.py --one WORKLOAD K --part-dir DIR
      one (workload, K) into DIR/WORKLOAD.K.json (for running Ks in parallel
      processes: at R-MAT scale 23 one K takes hours on one core);
  python tests/golden/make_digests.py --batch LO HI --part-dir DIR
      graphs LO..HI-1 of the batched workload into DIR/batch.LO-HI.json;
  python tests/golden/make_digests.py --merge DIR
      every part file of DIR into digests.json.
"""
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "digests.json")
BATCH = "chunglu-batch-4096"


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype).tobytes()).hexdigest()


def digests(rowptr, col, n2o, mask, sup):
    rows = np.repeat(np.arange(len(rowptr) - 1, dtype=np.int64), np.diff(rowptr))
    a = n2o[rows].astype(np.int64)
    b = n2o[col].astype(np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keep = mask.astype(bool)
    order = np.lexsort((hi[keep], lo[keep]))
    triples = np.stack([lo[keep][order], hi[keep][order], sup[keep][order].astype(np.int64)], axis=1)
    return {
        "mask_sha256": sha(mask, np.uint8),
        "support_sha256": sha(sup, "<i4"),
        "keyed_sha256": sha(triples, "<i8"),
        "truss_edges": int(keep.sum()),
        "support_sum": int(sup.astype(np.int64).sum()),
    }


def canonical(name):
    n, s, d = synth.workload_pairs(name)
    t0 = time.time()
    rowptr, col, n2o = oracle.canonical_csr(n, s, d, 1)
    print("%s: n=%d m=%d canonical in %.1fs" % (name, n, len(col), time.time() - t0), flush=True)
    return n, rowptr, col, n2o


def one(rowptr, col, n2o, K):
    t0 = time.time()
    mask, sup, rounds = oracle.truss(rowptr, col, K, "P")
    rec = {"rounds": int(rounds), **digests(rowptr, col, n2o, mask, sup)}
    print("  K=%d rounds=%d truss=%d in %.1fs" % (K, rounds, rec["truss_edges"], time.time() - t0), flush=True)
    return rec


def save(data):
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(OUT + ".tmp", OUT)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        n, rowptr, col, n2o = canonical(name)
        entry = data.get(name, {"n": n, "m": int(len(col)), "K": {}})
        for K in synth.WORKLOADS[name].Ks:
            if str(K) in entry["K"]:
                continue
            entry["K"][str(K)] = one(rowptr, col, n2o, K)
            data[name] = entry
            save(data)


def part_one(name, K, part_dir):
    n, rowptr, col, n2o = canonical(name)
    rec = {"workload": name, "n": n, "m": int(len(col)), "K": int(K), "result": one(rowptr, col, n2o, K)}
    path = os.path.join(part_dir, "%s.%d.json" % (name, K))
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(path + ".tmp", path)


def part_batch(lo, hi, part_dir):
    p = synth.WORKLOADS[BATCH].params
    out = {"lo": lo, "hi": hi, "graphs": []}
    t0 = time.time()
    for g in range(lo, hi):
        n, gamma, dbar, K = synth.batch_params(p["seed"], g, p["nmin"], p["nmax"])
        _, s, d = synth.chung_lu(n, gamma, dbar, p["seed"] * 1_000_003 + g)
        rowptr, col, _ = oracle.canonical_csr(n, s, d, 1)
        mask, sup, rounds = oracle.truss(rowptr, col, K, "P")
        out["graphs"].append({"n": n, "m": int(len(col)), "K": int(K), "rounds": int(rounds),
                              "truss_edges": int(mask.astype(np.int64).sum()),
                              "support_sum": int(sup.astype(np.int64).sum()),
                              "mask_sha256": sha(mask, np.uint8), "support_sha256": sha(sup, "<i4")})
        if (g - lo) % 64 == 63:
            print("  batch graphs %d..%d done in %.1fs" % (lo, g, time.time() - t0), flush=True)
    path = os.path.join(part_dir, "batch.%d-%d.json" % (lo, hi))
    with open(path + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(path + ".tmp", path)


def merge(part_dir):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for path in sorted(glob.glob(os.path.join(part_dir, "*.json"))):
        rec = json.load(open(path))
        if "workload" in rec:
            entry = data.setdefault(rec["workload"], {"n": rec["n"], "m": rec["m"], "K": {}})
            assert entry["n"] == rec["n"] and entry["m"] == rec["m"], path
            entry["K"][str(rec["K"])] = rec["result"]
    parts = sorted((json.load(open(p)) for p in glob.glob(os.path.join(part_dir, "batch.*.json"))),
                   key=lambda r: r["lo"])
    if parts:
        graphs = [g for r in parts for g in r["graphs"]]
        count = synth.WORKLOADS[BATCH].params["count"]
        assert [r["lo"] for r in parts] == sorted(set(r["lo"] for r in parts))
        assert len(graphs) == count and parts[0]["lo"] == 0 and parts[-1]["hi"] == count, "batch parts incomplete"
        hm, hs = hashlib.sha256(), hashlib.sha256()
        for g in graphs:
            hm.update(bytes.fromhex(g["mask_sha256"]))
            hs.update(bytes.fromhex(g["support_sha256"]))
        data[BATCH] = {"graphs": count, "m": int(sum(g["m"] for g in graphs)),
                       "n": int(sum(g["n"] for g in graphs)),
                       "K": [g["K"] for g in graphs], "rounds": [g["rounds"] for g in graphs],
                       "truss_edges": [g["truss_edges"] for g in graphs],
                       "support_sum": [g["support_sum"] for g in graphs],
                       "mask_sha256": hm.hexdigest(), "support_sha256": hs.hexdigest()}
    save(data)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args[:1] == ["--one"]:
        part_one(args[1], int(args[2]), args[args.index("--part-dir") + 1])
    elif args[:1] == ["--batch"]:
        part_batch(int(args[1]), int(args[2]), args[args.index("--part-dir") + 1])
    elif args[:1] == ["--merge"]:
        merge(args[1])
    else:
        main(args or ["rmat-s12-ef8", "rmat-s20-ef16"])
