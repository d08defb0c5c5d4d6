"""Writes tests/golden/digests.json: the oracle's K-truss results on the full-size
synthetic workloads, reduced to digests so that the GPU tests can compare bit
for bit without storing per-edge arrays.

Uses only the input generators (synth) and the CPU oracle (oracle/, mode P,
its own canonicalisation).  For each (workload, K):
  m, n, rounds, truss_edges, support_sum,
  mask_sha256     sha256 of the uint8 mask in canonical edge order,
  support_sha256  sha256 of the little-endian int32 supports in canonical order,
  keyed_sha256    sha256 of the survivors as little-endian int64 triples
                  (min original id, max original id, support), sorted.
The keyed digest does not depend on the relabelling, so a builder bug cannot
hide behind it.

Run:  python tests/golden/make_digests.py [workload ...]   (tens of minutes)
"""
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


def digests(rowptr, col, n2o, mask, sup):
    rows = np.repeat(np.arange(len(rowptr) - 1, dtype=np.int64), np.diff(rowptr))
    a = n2o[rows].astype(np.int64)
    b = n2o[col].astype(np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keep = mask.astype(bool)
    order = np.lexsort((hi[keep], lo[keep]))
    triples = np.stack([lo[keep][order], hi[keep][order], sup[keep][order].astype(np.int64)], axis=1)
    return {
        "mask_sha256": hashlib.sha256(np.ascontiguousarray(mask, np.uint8).tobytes()).hexdigest(),
        "support_sha256": hashlib.sha256(np.ascontiguousarray(sup, "<i4").tobytes()).hexdigest(),
        "keyed_sha256": hashlib.sha256(np.ascontiguousarray(triples, "<i8").tobytes()).hexdigest(),
        "truss_edges": int(keep.sum()),
        "support_sum": int(sup.astype(np.int64).sum()),
    }


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        w = synth.WORKLOADS[name]
        n, s, d = synth.workload_pairs(name)
        t0 = time.time()
        rowptr, col, n2o = oracle.canonical_csr(n, s, d, 1)
        print("%s: n=%d m=%d canonical in %.1fs" % (name, n, len(col), time.time() - t0), flush=True)
        entry = data.get(name, {"n": n, "m": int(len(col)), "K": {}})
        for K in w.Ks:
            if str(K) in entry["K"]:
                continue
            t0 = time.time()
            mask, sup, rounds = oracle.truss(rowptr, col, K, "P")
            rec = {"rounds": int(rounds), **digests(rowptr, col, n2o, mask, sup)}
            entry["K"][str(K)] = rec
            print("  K=%d rounds=%d truss=%d in %.1fs" % (K, rounds, rec["truss_edges"], time.time() - t0), flush=True)
            data[name] = entry
            with open(OUT + ".tmp", "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or ["rmat-s12-ef8", "rmat-s20-ef16"])
