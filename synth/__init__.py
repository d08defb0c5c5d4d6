"""Seeded synthetic inputs for the K-truss workloads.

Input generation only: every function returns raw, unordered vertex pairs
(``src``, ``dst`` as int32 NumPy arrays, possibly with self-loops and
duplicates) plus the vertex count.  Canonicalisation (dropping loops and
duplicates, relabelling, orienting) is NOT done here: the library's CSR builder
and the oracle each do it in their own code.

The paper measured SNAP graphs from the GraphChallenge collection, which are not
available here; the named workloads below are synthetic stand-ins with the same
character (power-law degree skew, a wide range of sizes, many small graphs).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (host code, no GPU)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, i64, u64, dbl, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, p, p]
        lib.synth_rmat.restype = ctypes.c_int
        lib.synth_distinct_vertices.argtypes = [i32, i32, u64, p]
        lib.synth_distinct_vertices.restype = ctypes.c_int
        lib.synth_chung_lu.argtypes = [i32, dbl, dbl, u64, p, p, i64]
        lib.synth_chung_lu.restype = i64
        lib.synth_batch_params.argtypes = [u64, i32, i32, i32, p, p, p, p]
        lib.synth_batch_params.restype = None
        lib.synth_ba.argtypes = [i32, i32, u64, p, p, i64]
        lib.synth_ba.restype = i64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int):
    """R-MAT pairs: 2^scale vertices, 2^scale*edge_factor pairs, no noise."""
    n = 1 << scale
    npairs = n * edge_factor
    src = np.empty(npairs, np.int32)
    dst = np.empty(npairs, np.int32)
    rc = _load().synth_rmat(scale, edge_factor, a, b, c, seed, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("synth_rmat failed: %d" % rc)
    return n, src, dst


def distinct_vertices(n: int, size: int, seed: int) -> np.ndarray:
    out = np.empty(size, np.int32)
    rc = _load().synth_distinct_vertices(n, size, seed, _ptr(out))
    if rc != 0:
        raise ValueError("synth_distinct_vertices failed: %d" % rc)
    return out


def clique_pairs(verts: np.ndarray):
    """All unordered pairs of `verts` (a planted clique)."""
    v = np.asarray(verts, np.int32)
    iu, ju = np.triu_indices(len(v), k=1)
    return v[iu].astype(np.int32), v[ju].astype(np.int32)


def chung_lu(n: int, gamma: float, dbar: float, seed: int):
    cap = int(round(n * dbar / 2.0)) + 1
    src = np.empty(cap, np.int32)
    dst = np.empty(cap, np.int32)
    k = _load().synth_chung_lu(n, gamma, dbar, seed, _ptr(src), _ptr(dst), cap)
    if k < 0:
        raise ValueError("synth_chung_lu failed: %d" % k)
    return n, src[:k].copy(), dst[:k].copy()


def batch_params(seed: int, g: int, nmin: int = 64, nmax: int = 20000):
    n = ctypes.c_int32()
    gamma = ctypes.c_double()
    dbar = ctypes.c_double()
    K = ctypes.c_int32()
    _load().synth_batch_params(seed, g, nmin, nmax, ctypes.addressof(n), ctypes.addressof(gamma),
                               ctypes.addressof(dbar), ctypes.addressof(K))
    return n.value, gamma.value, dbar.value, K.value


def barabasi_albert(n: int, m: int, seed: int):
    total = (m + 1) * m // 2 + (n - m - 1) * m
    src = np.empty(total, np.int32)
    dst = np.empty(total, np.int32)
    k = _load().synth_ba(n, m, seed, _ptr(src), _ptr(dst), total)
    if k != total:
        raise ValueError("synth_ba failed: %d" % k)
    return n, src, dst


def bipartite_chung_lu(nu: int, nv: int, gamma_u: float, gamma_v: float, npairs: int, seed: int):
    """Bipartite pairs (u in [0, nu), v in [0, nv)) with power-law expected
    degrees on both sides: each of the npairs draws picks u with probability
    proportional to (u + 1)^(-1 / (gamma_u - 1)) and v likewise with gamma_v
    (repeated pairs possible; the builders drop them).  Returns (nu, nv, u, v)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wu = (np.arange(nu, dtype=np.float64) + 1.0) ** (-1.0 / (gamma_u - 1.0))
    wv = (np.arange(nv, dtype=np.float64) + 1.0) ** (-1.0 / (gamma_v - 1.0))
    cu, cv = np.cumsum(wu), np.cumsum(wv)
    u = np.searchsorted(cu, rng.random(npairs) * cu[-1], side="right")
    v = np.searchsorted(cv, rng.random(npairs) * cv[-1], side="right")
    return nu, nv, np.minimum(u, nu - 1).astype(np.int32), np.minimum(v, nv - 1).astype(np.int32)


def bipartite_csr(nu: int, nv: int, u, v):
    """Rows over U with ascending, distinct columns (plain NumPy, for tests):
    (rowptr int32[nu+1], col int32[m])."""
    key = np.unique(np.asarray(u, np.int64) * nv + np.asarray(v, np.int64))
    rows, cols = key // nv, key % nv
    rowptr = np.zeros(nu + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32)


# ---------------------------------------------------------------- small graphs

def _pairs(edges, n):
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    return n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def complete(n: int):
    iu, ju = np.triu_indices(n, k=1)
    return n, iu.astype(np.int32), ju.astype(np.int32)


def path(n: int):
    return _pairs([(i, i + 1) for i in range(n - 1)], n)


def cycle(n: int):
    return _pairs([(i, (i + 1) % n) for i in range(n)], n)


def star(n: int):
    return _pairs([(0, i) for i in range(1, n)], n)


def grid(r: int, c: int):
    e = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                e.append((v, v + 1))
            if i + 1 < r:
                e.append((v, v + c))
    return _pairs(e, r * c)


def complete_bipartite(a: int, b: int):
    return _pairs([(i, a + j) for i in range(a) for j in range(b)], a + b)


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return _pairs(outer + spokes + inner, 10)


def erdos_renyi(n: int, p: float, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(len(iu)) < p
    return n, iu[keep].astype(np.int32), ju[keep].astype(np.int32)


def raw_noise(n: int, npairs: int, seed: int):
    """Uniform random pairs including self-loops and duplicates (builder tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return n, rng.integers(0, n, npairs).astype(np.int32), rng.integers(0, n, npairs).astype(np.int32)


def disjoint_union(*graphs):
    """Concatenate graphs (n, src, dst) with shifted vertex ids."""
    off = 0
    ss, dd = [], []
    for n, s, d in graphs:
        ss.append(s.astype(np.int64) + off)
        dd.append(d.astype(np.int64) + off)
        off += n
    return off, np.concatenate(ss).astype(np.int32), np.concatenate(dd).astype(np.int32)


# ---------------------------------------------------------------- named workloads

@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: how to make its pairs and which K values it runs."""
    name: str
    kind: str
    params: dict = field(default_factory=dict)
    Ks: tuple = ()


WORKLOADS = {
    # small R-MAT the oracle finishes in well under a second
    "rmat-s12-ef8": Workload("rmat-s12-ef8", "rmat",
                             dict(scale=12, edge_factor=8, abc=(0.57, 0.19, 0.19), seed=1), (3, 4, 5, 6)),
    # R-MAT at the size of the paper's largest graph (cit-Patents, 16.5M edges)
    "rmat-s20-ef16": Workload("rmat-s20-ef16", "rmat",
                              dict(scale=20, edge_factor=16, abc=(0.57, 0.19, 0.19), seed=2), (3, 5, 8, 12)),
    # high-skew stress: R-MAT scale 23 plus a planted 600-clique on random vertices
    "rmat-s23-ef16-clique600": Workload("rmat-s23-ef16-clique600", "rmat+clique",
                                        dict(scale=23, edge_factor=16, abc=(0.65, 0.15, 0.15), seed=3,
                                             clique=600, clique_seed=4), (3, 10, 50, 600)),
    # learned-scheduler evaluation graphs
    "rmat-s22-ef16": Workload("rmat-s22-ef16", "rmat",
                              dict(scale=22, edge_factor=16, abc=(0.6, 0.2, 0.15), seed=22), (3, 6, 10)),
    "ba-4M-m8": Workload("ba-4M-m8", "ba", dict(n=4 * 1024 * 1024, m=8, seed=23), (3, 6, 10)),
    # bipartite graph for butterfly counting: power-law degrees on both sides
    "bip-cl-1M-16M": Workload("bip-cl-1M-16M", "bipartite",
                              dict(nu=1 << 20, nv=1 << 18, gamma_u=2.5, gamma_v=2.2, pairs=16 << 20, seed=31)),
    # many small graphs of uneven sizes in one batched run (K per graph in 3..8)
    "chunglu-batch-4096": Workload("chunglu-batch-4096", "batch", dict(count=4096, seed=5, nmin=64, nmax=20000)),
}


def workload_pairs(name: str):
    """(n, src, dst) for a named single-graph workload."""
    w = WORKLOADS[name]
    p = w.params
    if w.kind in ("rmat", "rmat+clique"):
        a, b, c = p["abc"]
        n, s, d = rmat(p["scale"], p["edge_factor"], a, b, c, p["seed"])
        if w.kind == "rmat+clique":
            cs, cd = clique_pairs(distinct_vertices(n, p["clique"], p["clique_seed"]))
            s = np.concatenate([s, cs])
            d = np.concatenate([d, cd])
        return n, s, d
    if w.kind == "ba":
        return barabasi_albert(p["n"], p["m"], p["seed"])
    raise KeyError(name)


def bipartite_pairs(name: str):
    """(nu, nv, u, v) for a named bipartite workload."""
    p = WORKLOADS[name].params
    return bipartite_chung_lu(p["nu"], p["nv"], p["gamma_u"], p["gamma_v"], p["pairs"], p["seed"])


def batch_graphs(count: int = 4096, seed: int = 5, nmin: int = 64, nmax: int = 20000, threads: int = 16):
    """The many-small-graphs workload: a list of (n, src, dst, K) Chung-Lu graphs.

    Graph g has n log-uniform in [nmin, nmax], power-law exponent uniform in
    [2.1, 3.0], mean degree uniform in [4, 64] and K uniform in {3..8}, all drawn
    from (seed, g); its pairs use seed * 1000003 + g.  Generated on `threads`
    threads (the C generator runs outside the interpreter lock); the result does
    not depend on the thread count."""
    from concurrent.futures import ThreadPoolExecutor

    def one(g):
        n, gamma, dbar, K = batch_params(seed, g, nmin, nmax)
        _, s, d = chung_lu(n, gamma, dbar, seed * 1_000_003 + g)
        return n, s, d, K

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(count)))
