"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, library routines (SciPy sparse products, networkx.k_truss),
brute force and exhaustive search on tiny graphs, and invariants of the truss.

Each pin is chosen so that a plausible slip in the oracle (a dropped triangle
corner, a wrong threshold direction, a transposed operand, an off-by-one in the
pass count) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def csr_of(g, order=1):
    n, s, d = g
    rp, col, n2o = oracle.canonical_csr(n, s, d, order)
    return n, rp, col, n2o


def sym_matrix(n, rp, col):
    rows = np.repeat(np.arange(n), np.diff(rp))
    A = sp.csr_matrix((np.ones(len(col), np.int64), (rows, col)), shape=(n, n))
    return (A + A.T).tocsr(), rows


def scipy_supports(n, rp, col):
    """Round-one supports from the plain definition S = (A A) o A on the symmetric adjacency."""
    A, rows = sym_matrix(n, rp, col)
    S = (A @ A).multiply(A).tocsr()
    return np.asarray(S[rows, col]).ravel().astype(np.int64)


def original_keys(rp, col, n2o):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    a, b = n2o[rows].astype(np.int64), n2o[col].astype(np.int64)
    return np.minimum(a, b) * (1 << 32) + np.maximum(a, b)


MODES = ("R", "P")


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [3, 4, 5, 7, 9])
@pytest.mark.parametrize("mode", MODES)
def test_complete_graph(n, mode):
    _, rp, col, _ = csr_of(synth.complete(n))
    assert len(col) == n * (n - 1) // 2
    for K in range(2, n + 3):
        mask, sup, rounds = oracle.truss(rp, col, K, mode)
        if K <= n:       # K_n is its own n-truss: every edge lies in n-2 triangles
            assert mask.all() and (sup == n - 2).all() and rounds == 1
        else:            # one pass removes everything, a second finds nothing to remove
            assert not mask.any() and not sup.any() and rounds == 2


@pytest.mark.parametrize("g", [synth.path(7), synth.star(9), synth.cycle(8), synth.cycle(5),
                               synth.complete_bipartite(3, 4), synth.petersen(), synth.grid(4, 5)])
@pytest.mark.parametrize("mode", MODES)
def test_triangle_free(g, mode):
    _, rp, col, _ = csr_of(g)
    assert (oracle.supports(rp, col) == 0).all()
    mask, sup, rounds = oracle.truss(rp, col, 3, mode)
    assert not mask.any() and rounds == 2
    mask, sup, rounds = oracle.truss(rp, col, 2, mode)
    assert mask.all() and rounds == 1


@pytest.mark.parametrize("mode", MODES)
def test_empty_graph(mode):
    rp = np.zeros(6, np.int32)
    col = np.zeros(0, np.int32)
    for K in (2, 3, 10):
        mask, sup, rounds = oracle.truss(rp, col, K, mode)
        assert len(mask) == 0 and rounds == 1


@pytest.mark.parametrize("mode", MODES)
def test_bridge_between_two_k4(mode):
    # two K4 joined by one edge: the bridge lies in no triangle
    e = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    e += [(a + 4, b + 4) for a, b in e] + [(3, 4)]
    g = (8, np.array([x for x, _ in e], np.int32), np.array([y for _, y in e], np.int32))
    n, rp, col, n2o = csr_of(g, order=0)
    mask, sup, rounds = oracle.truss(rp, col, 4, mode)
    keys = original_keys(rp, col, n2o)
    bridge = keys == (3 << 32) + 4
    assert mask[~bridge].all() and not mask[bridge].any()
    assert (sup[~bridge] == 2).all() and rounds == 2


# ----------------------------------------------------- library definitions

@pytest.mark.parametrize("g", ["rmat12", "er"])
def test_round_one_supports_match_scipy(g, rmat12):
    graph = rmat12 if g == "rmat12" else synth.erdos_renyi(300, 0.08, 11)
    n, rp, col, _ = csr_of(graph)
    ours = oracle.supports(rp, col).astype(np.int64)
    assert np.array_equal(ours, scipy_supports(n, rp, col))


def test_support_sum_is_three_triangles(rmat12):
    n, rp, col, _ = csr_of(rmat12)
    A, _ = sym_matrix(n, rp, col)
    triangles6 = int((A @ A).multiply(A).sum())      # trace(A^3) = 6 * triangles
    assert triangles6 % 6 == 0
    assert int(oracle.supports(rp, col).sum()) == 3 * (triangles6 // 6)
    import networkx as nx
    G = nx.Graph()
    G.add_edges_from(zip(np.repeat(np.arange(n), np.diff(rp)).tolist(), col.tolist()))
    assert sum(nx.triangles(G).values()) == 3 * (triangles6 // 6)


@pytest.mark.parametrize("scale", [12, 14])
@pytest.mark.parametrize("mode", MODES)
def test_k3_closed_form(scale, mode):
    # For K=3 the removed edges lie in no triangle, so no other support changes:
    # T3 = {S1 >= 1} with supports S1, in at most two passes.
    n, rp, col, _ = csr_of(synth.rmat(scale, 8, 0.57, 0.19, 0.19, 7 + scale))
    S1 = scipy_supports(n, rp, col)
    mask, sup, rounds = oracle.truss(rp, col, 3, mode)
    assert np.array_equal(mask.astype(bool), S1 >= 1)
    assert np.array_equal(sup.astype(np.int64), np.where(S1 >= 1, S1, 0))
    assert rounds == (2 if (S1 == 0).any() else 1)


@pytest.mark.parametrize("K", [3, 4, 5, 6, 8, 12])
def test_truss_matches_networkx(K, rmat12):
    import networkx as nx
    n, rp, col, n2o = csr_of(rmat12)
    s, d = rmat12[1], rmat12[2]
    G = nx.Graph()
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    T = nx.k_truss(G, K)
    want = np.array(sorted(min(a, b) * (1 << 32) + max(a, b) for a, b in T.edges()), np.int64)
    mask, sup, rounds = oracle.truss(rp, col, K, "P")
    got = np.sort(original_keys(rp, col, n2o)[mask.astype(bool)])
    assert np.array_equal(got, want)


# --------------------------------------------- brute force and exhaustive

def random_small(seed, n, p):
    n, s, d = synth.erdos_renyi(n, p, seed)
    rp, col, _ = oracle.canonical_csr(n, s, d, 0)
    return n, rp, col


@pytest.mark.parametrize("seed", range(12))
def test_exhaustive_maximality(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 8))
    p = float(rng.uniform(0.5, 0.9))
    n, rp, col = random_small(seed, n, p)
    if len(col) > 16:
        col_keep = 16
        # trim to the first 16 edges of a fresh CSR so the 2^m search stays small
        e = oracle.edges_of(rp, col)[:col_keep]
        g = (n, np.array([a for a, _ in e], np.int32), np.array([b for _, b in e], np.int32))
        rp, col, _ = oracle.canonical_csr(*g, 0)
    edges = oracle.edges_of(rp, col)
    for K in (3, 4, 5):
        want = oracle.truss_exhaustive(n, edges, K)
        for mode in MODES:
            mask, _, _ = oracle.truss(rp, col, K, mode)
            assert list(mask) == want, (seed, K, mode)


@pytest.mark.parametrize("seed", range(8))
def test_bruteforce_tier_agrees(seed):
    rng = np.random.default_rng(100 + seed)
    n, rp, col = random_small(100 + seed, int(rng.integers(12, 30)), float(rng.uniform(0.15, 0.5)))
    edges = oracle.edges_of(rp, col)
    for K in (3, 4, 5, 6):
        bmask, bsup, brounds = oracle.truss_bruteforce(n, edges, K)
        for mode in MODES:
            mask, sup, rounds = oracle.truss(rp, col, K, mode)
            assert list(mask) == bmask and list(sup) == bsup and rounds == brounds, (seed, K, mode)


@pytest.mark.parametrize("seed", range(6))
def test_modes_agree_on_rmat(seed):
    n, rp, col, _ = csr_of(synth.rmat(11, 12, 0.6, 0.15, 0.15, 200 + seed))
    for K in (3, 4, 6, 9, 15):
        a = oracle.truss(rp, col, K, "R")
        b = oracle.truss(rp, col, K, "P")
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("K", [3, 4, 5, 6, 8, 12])
def test_survivors_recount(K, rmat12):
    _, rp, col, _ = csr_of(rmat12)
    mask, sup, _ = oracle.truss(rp, col, K, "P")
    recount = oracle.supports(rp, col, mask)
    assert np.array_equal(recount, sup)
    assert (sup[mask.astype(bool)] >= K - 2).all()
    assert (sup[~mask.astype(bool)] == 0).all()


def test_nested_trusses(rmat12):
    _, rp, col, _ = csr_of(rmat12)
    prev = None
    for K in range(2, 20):
        mask, _, _ = oracle.truss(rp, col, K, "P")
        if prev is not None:
            assert not (mask & ~prev).any()
        prev = mask


def test_permutation_invariance(rmat12):
    n, s, d = rmat12
    perm = np.random.default_rng(3).permutation(n).astype(np.int32)
    _, rp, col, n2o = csr_of(rmat12)
    _, rp2, col2, n2o2 = csr_of((n, perm[s], perm[d]))
    inv = np.argsort(perm).astype(np.int32)
    for K in (3, 5, 7):
        m1, s1, r1 = oracle.truss(rp, col, K, "P")
        m2, s2, r2 = oracle.truss(rp2, col2, K, "P")
        k1 = original_keys(rp, col, n2o)
        k2 = original_keys(rp2, col2, inv[n2o2])
        o1, o2 = np.argsort(k1), np.argsort(k2)
        assert np.array_equal(k1[o1], k2[o2])
        assert np.array_equal(m1[o1], m2[o2]) and np.array_equal(s1[o1], s2[o2]) and r1 == r2


def test_disjoint_union(rmat12):
    g1 = rmat12
    g2 = synth.rmat(10, 10, 0.6, 0.15, 0.15, 99)
    gu = synth.disjoint_union(g1, g2)
    for K in (3, 5, 8):
        parts = []
        for g, off in ((g1, 0), (g2, g1[0])):
            _, rp, col, n2o = csr_of(g)
            mask, sup, r = oracle.truss(rp, col, K, "P")
            keys = original_keys(rp, col, (n2o + off).astype(np.int32))
            parts.append((keys[mask.astype(bool)], sup[mask.astype(bool)], r))
        _, rp, col, n2o = csr_of(gu)
        mask, sup, r = oracle.truss(rp, col, K, "P")
        keys = original_keys(rp, col, n2o)
        want_k = np.concatenate([p[0] for p in parts])
        want_s = np.concatenate([p[1] for p in parts])
        o = np.argsort(want_k)
        got = mask.astype(bool)
        og = np.argsort(keys[got])
        assert np.array_equal(keys[got][og], want_k[o]) and np.array_equal(sup[got][og], want_s[o])
        assert r == max(parts[0][2], parts[1][2])


def test_planted_clique_survives():
    n, s, d = synth.rmat(12, 4, 0.57, 0.19, 0.19, 5)
    verts = synth.distinct_vertices(n, 40, 6)
    cs, cd = synth.clique_pairs(verts)
    g = (n, np.concatenate([s, cs]), np.concatenate([d, cd]))
    _, rp, col, n2o = csr_of(g)
    mask, sup, _ = oracle.truss(rp, col, 40, "P")
    keys = set(original_keys(rp, col, n2o)[mask.astype(bool)].tolist())
    clique = {min(a, b) * (1 << 32) + max(a, b) for a, b in zip(cs.tolist(), cd.tolist())}
    assert clique <= keys


@pytest.mark.parametrize("K", [4, 6])
def test_restart_from_intermediate_mask(K, rmat12):
    _, rp, col, _ = csr_of(rmat12)
    mask, sup, _ = oracle.truss(rp, col, K, "P")
    rng = np.random.default_rng(K)
    start = (mask.astype(bool) | (rng.random(len(col)) < 0.5)).astype(np.uint8)
    for mode in MODES:
        m2, s2, _ = oracle.truss(rp, col, K, mode, alive_init=start)
        assert np.array_equal(m2, mask) and np.array_equal(s2, sup)
    # a K+1 run started from the K-truss gives the K+1 truss
    m3, s3, _ = oracle.truss(rp, col, K + 1, "P", alive_init=mask)
    m4, s4, _ = oracle.truss(rp, col, K + 1, "P")
    assert np.array_equal(m3, m4) and np.array_equal(s3, s4)


def test_prune_definition():
    sup = np.array([0, 1, 2, 3, 5, 0], np.int32)
    alive = np.array([1, 1, 1, 1, 1, 0], np.uint8)
    new, removed = oracle.prune(sup, alive, 4)   # keep support >= 2
    assert list(new) == [0, 0, 1, 1, 1, 0] and removed == 2


# ------------------------------------------------------ canonical CSR input

def test_canonical_csr_properties():
    n, s, d = synth.raw_noise(300, 3000, 4)
    for order in (0, 1, 2):
        rp, col, n2o = oracle.canonical_csr(n, s, d, order)
        assert sorted(n2o.tolist()) == list(range(n))
        rows = np.repeat(np.arange(n), np.diff(rp))
        assert (col > rows).all()
        assert all((np.diff(col[rp[i]:rp[i + 1]]) > 0).all() for i in range(n))
        want = {(min(a, b), max(a, b)) for a, b in zip(s.tolist(), d.tolist()) if a != b}
        got = {(min(n2o[a], n2o[b]), max(n2o[a], n2o[b])) for a, b in zip(rows.tolist(), col.tolist())}
        assert got == want
        deg = np.bincount(np.concatenate([rows, col]), minlength=n)
        if order == 1:
            assert (np.diff(deg) >= 0).all()
        if order == 2:
            assert (np.diff(deg) <= 0).all()
        if order == 0:
            assert (n2o == np.arange(n)).all()


def test_canonical_relabel_tie_break():
    """Equal-degree vertices take consecutive new labels in ascending original
    id (ascending order), and in ascending original id too under the
    descending order: the relabelling is the stable sort of the vertices by
    degree.  A hand-made graph whose degree classes interleave the ids."""
    # degrees by original id: 0:1 1:3 2:1 3:2 4:3 5:2 6:0 7:2 (stars and paths)
    pairs = [(1, 0), (1, 2), (1, 3), (4, 3), (4, 5), (4, 7), (5, 7)]
    s = np.array([a for a, _ in pairs], np.int32)
    d = np.array([b for _, b in pairs], np.int32)
    _, _, n2o_up = oracle.canonical_csr(8, s, d, 1)
    assert n2o_up.tolist() == [6, 0, 2, 3, 5, 7, 1, 4]
    _, _, n2o_down = oracle.canonical_csr(8, s, d, 2)
    assert n2o_down.tolist() == [1, 4, 3, 5, 7, 0, 2, 6]
    # the same rule on a random graph, written as a stable sort by degree
    n, rs, rd = synth.raw_noise(400, 1500, 11)
    keep = rs != rd
    deg = np.zeros(n, np.int64)
    e = {(min(a, b), max(a, b)) for a, b in zip(rs[keep].tolist(), rd[keep].tolist())}
    for a, b in e:
        deg[a] += 1
        deg[b] += 1
    assert oracle.canonical_csr(n, rs, rd, 1)[2].tolist() == np.argsort(deg, kind="stable").tolist()
    assert oracle.canonical_csr(n, rs, rd, 2)[2].tolist() == np.argsort(-deg, kind="stable").tolist()


def test_supports_of_listed_edges_match_scipy(rmat12):
    """The listed-edge support evaluation (used to time the oracle on a sample
    of a large graph) equals SciPy's (A A) o A at those edges."""
    n, s, d = rmat12
    rp, col, _ = oracle.canonical_csr(n, s, d)
    m = len(col)
    rows = np.repeat(np.arange(n), np.diff(rp))
    A = sp.coo_matrix((np.ones(m, np.int64), (rows, col)), shape=(n, n)).tocsr()
    A = A + A.T
    S = (A @ A).multiply(A).tocsr()
    edges = np.random.default_rng(3).choice(m, 500, replace=False)
    got, secs = oracle.supports_of(rp, col, edges, timed=True)
    want = np.asarray(S[rows[edges], col[edges]]).ravel()
    assert np.array_equal(got, want) and secs >= 0.0
    assert len(oracle.supports_of(rp, col, np.zeros(0, np.int64))) == 0
