"""Pins of the butterfly oracle (CPU): closed forms, brute force over all
4-tuples, and the matrix identity count(u, v) = (B B^T B)[u, v] - deg(u) -
deg(v) + 1 on the edges of the biadjacency B (SciPy), with the total equal to
the sum over pairs of C(common neighbours, 2) and to the edge counts over 4."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def edges_to_csr(nu, nv, edges):
    u = np.array([a for a, _ in edges], np.int64)
    v = np.array([b for _, b in edges], np.int64)
    return synth.bipartite_csr(nu, nv, u, v)


def csr_edges(rp, col):
    return [(u, int(col[e])) for u in range(len(rp) - 1) for e in range(rp[u], rp[u + 1])]


@pytest.mark.parametrize("a,b", [(2, 2), (3, 4), (5, 2), (6, 7), (1, 9)])
def test_complete_bipartite(a, b):
    rp, col = edges_to_csr(a, b, [(u, v) for u in range(a) for v in range(b)])
    cnt, tot = oracle.butterflies(a, b, rp, col)
    assert tot == (a * (a - 1) // 2) * (b * (b - 1) // 2)
    assert (cnt == (a - 1) * (b - 1)).all()


def test_cycles_trees_and_empty():
    # C4: one butterfly; C6, C8 (even cycles longer than 4): none
    for k in (2, 3, 4):
        edges = [(i, i) for i in range(k)] + [(i, (i + 1) % k) for i in range(k)]
        rp, col = edges_to_csr(k, k, edges)
        cnt, tot = oracle.butterflies(k, k, rp, col)
        assert tot == (1 if k == 2 else 0) and (cnt == (1 if k == 2 else 0)).all()
    # a star and a path (trees): none
    for edges, nu, nv in (([(0, v) for v in range(6)], 1, 6), ([(0, 0), (1, 0), (1, 1), (2, 1)], 3, 2)):
        rp, col = edges_to_csr(nu, nv, edges)
        cnt, tot = oracle.butterflies(nu, nv, rp, col)
        assert tot == 0 and (cnt == 0).all()
    cnt, tot = oracle.butterflies(4, 3, np.zeros(5, np.int32), np.zeros(0, np.int32))
    assert tot == 0 and len(cnt) == 0


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_tiny(seed):
    rng = np.random.default_rng(seed)
    nu, nv = int(rng.integers(2, 7)), int(rng.integers(2, 7))
    edges = [(u, v) for u in range(nu) for v in range(nv) if rng.random() < 0.55]
    rp, col = edges_to_csr(nu, nv, edges)
    es = csr_edges(rp, col)
    want, want_tot = oracle.butterflies_bruteforce(nu, nv, es)
    cnt, tot = oracle.butterflies(nu, nv, rp, col)
    assert tot == want_tot and cnt.tolist() == want


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_matrix_identity(seed):
    nu, nv, u, v = synth.bipartite_chung_lu(3000, 1000, 2.4, 2.2, 20000, seed)
    rp, col = synth.bipartite_csr(nu, nv, u, v)
    rows = np.repeat(np.arange(nu), np.diff(rp))
    B = sp.csr_matrix((np.ones(len(col), np.int64), (rows, col)), shape=(nu, nv))
    BBB = (B @ B.T @ B).tocsr()
    du = np.diff(rp).astype(np.int64)
    dv = np.bincount(col, minlength=nv).astype(np.int64)
    want = np.asarray(BBB[rows, col]).ravel() - du[rows] - dv[col] + 1
    cnt, tot = oracle.butterflies(nu, nv, rp, col)
    assert np.array_equal(cnt, want)
    W = (B @ B.T).tocoo()
    off = W.row < W.col
    c = W.data[off].astype(np.int64)
    assert tot == int((c * (c - 1) // 2).sum()) and 4 * tot == int(cnt.sum())


def test_relabelling_invariance():
    nu, nv, u, v = synth.bipartite_chung_lu(500, 300, 2.3, 2.3, 4000, 9)
    rp, col = synth.bipartite_csr(nu, nv, u, v)
    cnt, tot = oracle.butterflies(nu, nv, rp, col)
    pu = np.random.default_rng(0).permutation(nu)
    pv = np.random.default_rng(1).permutation(nv)
    es = csr_edges(rp, col)
    rp2, col2 = synth.bipartite_csr(nu, nv, pu[[a for a, _ in es]], pv[[b for _, b in es]])
    cnt2, tot2 = oracle.butterflies(nu, nv, rp2, col2)
    assert tot2 == tot
    key = {(pu[a], pv[b]): int(c) for (a, b), c in zip(es, cnt)}
    assert all(key[e] == int(c) for e, c in zip(csr_edges(rp2, col2), cnt2))
    # swapping the sides leaves every edge's count
    rpt, colt = synth.bipartite_csr(nv, nu, [b for _, b in es], [a for a, _ in es])
    cntt, tott = oracle.butterflies(nv, nu, rpt, colt)
    keyt = {(a, b): int(c) for (b, a), c in zip(csr_edges(rpt, colt), cntt)}
    assert tott == tot and all(keyt[e] == int(c) for e, c in zip(es, cnt))
