"""K-truss ORACLE — test infrastructure only.

Plain, slow, obviously-correct CPU implementations of what the GPU library
computes, written from the paper (Blanco, Low, Kim, HPEC 2019).  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
package; the product path never does, and this package never imports the
product package.

Tiers:
  * ``ktruss_oracle.c`` (loaded via ctypes): canonical CSR from raw pairs;
    one support evaluation (of every edge, or of listed edges); the truss by
    literal Algorithm 1 recompute (mode "R") and by level-synchronous peeling
    (mode "P").
  * pure-Python brute force for tiny graphs (every vertex tested as the third
    corner of every edge) and exhaustive maximality over all edge subsets.
  * ``butterfly_oracle.c``: butterflies (4-cycles) of a bipartite graph per
    edge and in total, from the common-neighbour definition; a pure-Python
    brute force over all 4-tuples for tiny graphs.
  * ``mlp`` (float64 NumPy): the cost-model network's forward, backward and
    optimizer step, checked by finite differences in the tests.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ktruss_oracle.c")
_SRC_BFLY = os.path.join(_HERE, "butterfly_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain C99, -O2, no vectorisation pragmas)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", _SRC, _SRC_BFLY, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.orc_canonical_csr.argtypes = [p, p, i64, i32, i32, p, p, i64, p, p]
        lib.orc_supports.argtypes = [i32, p, p, p, p]
        lib.orc_truss_recompute.argtypes = [i32, p, p, i32, p, p, p, p]
        lib.orc_truss_peel.argtypes = [i32, p, p, i32, p, p, p, p]
        lib.orc_supports_of.argtypes = [i32, p, p, p, i64, p, p]
        lib.orc_butterflies.argtypes = [i32, i32, p, p, p, p]
        for f in (lib.orc_canonical_csr, lib.orc_supports, lib.orc_truss_recompute, lib.orc_truss_peel,
                  lib.orc_supports_of, lib.orc_butterflies):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


class OracleError(RuntimeError):
    pass


def canonical_csr(n, src, dst, order: int = 1):
    """Upper-triangular CSR (rowptr int32[n+1], col int32[m]) and new_to_old int32[n].

    order: 0 keep ids, 1 ascending degree (ties by old id), 2 descending degree.
    """
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    rowptr = np.zeros(n + 1, np.int32)
    col = np.zeros(max(len(src), 1), np.int32)
    n2o = np.zeros(max(n, 1), np.int32)
    m = ctypes.c_int64()
    rc = _load().orc_canonical_csr(_p(src), _p(dst), len(src), n, order, _p(rowptr), _p(col),
                                   len(col), _p(n2o), ctypes.addressof(m))
    if rc != 0:
        raise OracleError("orc_canonical_csr: %d" % rc)
    return rowptr, col[: m.value].copy(), n2o[:n].copy()


def supports(rowptr, col, alive=None):
    """One support evaluation: triangles of the alive subgraph per edge, 0 if dead."""
    n = len(rowptr) - 1
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    out = np.zeros(max(len(col), 1), np.int32)
    al = None if alive is None else np.ascontiguousarray(alive, np.uint8)
    rc = _load().orc_supports(n, _p(rowptr), _p(col), _p(al), _p(out))
    if rc != 0:
        raise OracleError("orc_supports: %d" % rc)
    return out[: len(col)]


def supports_of(rowptr, col, edges, timed: bool = False):
    """Supports (triangles containing the edge, whole graph alive) of the listed
    edge positions; with timed=True also the seconds of the per-edge loop."""
    n = len(rowptr) - 1
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    edges = np.ascontiguousarray(edges, np.int64)
    out = np.zeros(max(len(edges), 1), np.int32)
    ns = ctypes.c_int64()
    rc = _load().orc_supports_of(n, _p(rowptr), _p(col), _p(edges), len(edges), _p(out), ctypes.addressof(ns))
    if rc != 0:
        raise OracleError("orc_supports_of: %d" % rc)
    return (out[: len(edges)], ns.value * 1e-9) if timed else out[: len(edges)]


def truss(rowptr, col, K: int, mode: str = "P", alive_init=None):
    """(mask uint8[m], support int32[m], rounds) of the K-truss by mode "R" or "P"."""
    n = len(rowptr) - 1
    m = len(col)
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    mask = np.zeros(max(m, 1), np.uint8)
    sup = np.zeros(max(m, 1), np.int32)
    rounds = ctypes.c_int32()
    al = None if alive_init is None else np.ascontiguousarray(alive_init, np.uint8)
    f = {"R": _load().orc_truss_recompute, "P": _load().orc_truss_peel}[mode]
    rc = f(n, _p(rowptr), _p(col), int(K), _p(al), _p(mask), _p(sup), ctypes.addressof(rounds))
    if rc != 0:
        raise OracleError("orc_truss_%s: %d" % (mode, rc))
    return mask[:m], sup[:m], rounds.value


def butterflies(nu: int, nv: int, rowptr, col):
    """Butterflies (4-cycles) of a bipartite graph given as CSR rows over U with
    columns in [0, nv): (count int64[m] per edge, total)."""
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    count = np.zeros(max(len(col), 1), np.int64)
    total = ctypes.c_int64()
    rc = _load().orc_butterflies(int(nu), int(nv), _p(rowptr), _p(col), _p(count), ctypes.addressof(total))
    if rc != 0:
        raise OracleError("orc_butterflies: %d" % rc)
    return count[: len(col)], total.value


def butterflies_bruteforce(nu: int, nv: int, edges):
    """Every 4-tuple u1 < u2, v1 < v2 tried against the edge set (tiny graphs).
    edges: list of (u, v).  Returns (count per edge in the given order, total)."""
    es = set(edges)
    cnt = {e: 0 for e in edges}
    total = 0
    for u1 in range(nu):
        for u2 in range(u1 + 1, nu):
            for v1 in range(nv):
                for v2 in range(v1 + 1, nv):
                    quad = [(u1, v1), (u1, v2), (u2, v1), (u2, v2)]
                    if all(q in es for q in quad):
                        total += 1
                        for q in quad:
                            cnt[q] += 1
    return [cnt[e] for e in edges], total


def prune(support, alive, K: int):
    """Algorithm 1's mask and update lines: keep alive edges with support >= K-2.

    Returns (new alive uint8[m], number of edges removed)."""
    support = np.asarray(support, np.int64)
    alive = np.asarray(alive, np.uint8)
    keep = (alive != 0) & (support >= K - 2)
    return keep.astype(np.uint8), int((alive != 0).sum() - keep.sum())


# ------------------------------------------------------------ pure-Python tier

def edges_of(rowptr, col):
    """List of (u, v) with u < v in CSR order."""
    out = []
    for u in range(len(rowptr) - 1):
        for e in range(rowptr[u], rowptr[u + 1]):
            out.append((u, int(col[e])))
    return out


def truss_bruteforce(n: int, edges, K: int):
    """Algorithm 1 by brute force on a small graph given as a list of (u, v), u < v.

    Each pass counts, for every alive edge (u, v), the vertices w adjacent to both
    u and v through alive edges.  Returns (mask list, support list, rounds)."""
    m = len(edges)
    alive = [True] * m
    index = {e: i for i, e in enumerate(edges)}

    def adj(a, b):
        if a == b:
            return None
        key = (a, b) if a < b else (b, a)
        return index.get(key)

    rounds = 0
    while True:
        rounds += 1
        S = [0] * m
        for i, (u, v) in enumerate(edges):
            if not alive[i]:
                continue
            c = 0
            for w in range(n):
                e1, e2 = adj(u, w), adj(v, w)
                if e1 is not None and e2 is not None and alive[e1] and alive[e2]:
                    c += 1
            S[i] = c
        drop = [i for i in range(m) if alive[i] and S[i] < K - 2]
        if not drop:
            break
        for i in drop:
            alive[i] = False
    return [int(a) for a in alive], [S[i] if alive[i] else 0 for i in range(m)], rounds


def truss_exhaustive(n: int, edges, K: int):
    """The K-truss as the union of every edge subset in which each edge lies in
    >= K-2 triangles of that subset (the definition in Section I), by trying all
    2^m subsets.  For m <= ~18.  Returns the mask as a list of 0/1."""
    m = len(edges)
    index = {e: i for i, e in enumerate(edges)}
    tris = []
    for (u, v), i in index.items():
        for w in range(v + 1, n):
            j, k = index.get((u, w)), index.get((v, w))
            if j is not None and k is not None:
                tris.append((i, j, k))
    subsets = np.arange(1 << m, dtype=np.int64)
    cnt = np.zeros((m, 1 << m), np.int32)
    for (i, j, k) in tris:
        full = ((subsets >> i) & 1) & ((subsets >> j) & 1) & ((subsets >> k) & 1)
        cnt[i] += full.astype(np.int32)
        cnt[j] += full.astype(np.int32)
        cnt[k] += full.astype(np.int32)
    ok = np.ones(1 << m, bool)
    for i in range(m):
        member = ((subsets >> i) & 1).astype(bool)
        ok &= ~member | (cnt[i] >= K - 2)
    union = 0
    for s in subsets[ok]:
        union |= int(s)
    return [(union >> i) & 1 for i in range(m)]


def subsets_count(m: int) -> int:
    return 1 << m


def all_pairs(n: int):
    return list(itertools.combinations(range(n), 2))
