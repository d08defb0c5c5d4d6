"""Truss decomposition on the GPU against the oracle: every edge's trussness
is the largest K whose K-truss (the oracle's, K = 3, 4, ... until empty)
holds it, 2 for edges in no triangle; k_max is the largest K with a non-empty
truss.  Bit for bit, under every schedule."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def oracle_trussness(rp, col):
    m = len(col)
    t = np.full(m, 2, np.int32)
    if m == 0:
        return t, 0
    K = 3
    while True:
        mask, _, _ = oracle.truss(rp, col, K, "P")
        if not mask.any():
            return t, K - 1
        t[mask.astype(bool)] = K
        K += 1


GRAPHS = {
    "K7": synth.complete(7), "petersen": synth.petersen(), "path": synth.path(9),
    "two-K5": synth.disjoint_union(synth.complete(5), synth.complete(5)),
    "er": synth.erdos_renyi(80, 0.25, 3), "empty": (5, np.zeros(0, np.int32), np.zeros(0, np.int32)),
}


def run(rp, col, schedule):
    import torch
    g = kt().Graph(rp, col, device="cuda")
    t = kt().ktruss_tuning()
    t.plain_max_work = -1
    kt().ktruss_set_schedule(g, schedule, None, t)
    tr, kmax = kt().ktruss_decompose(g)
    torch.cuda.synchronize()
    return tr.cpu().numpy(), kmax


@pytest.mark.parametrize("schedule", [0, 1, 4, 5])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_small_graphs(name, schedule):
    n, s, d = GRAPHS[name]
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    print("case decompose %s schedule=%d m=%d" % (name, schedule, len(col)), flush=True)
    want, want_k = oracle_trussness(rp, col)
    got, got_k = run(rp, col, schedule)
    assert np.array_equal(got, want) and got_k == want_k, (name, got_k, want_k)


@pytest.mark.parametrize("schedule", [0, 1, 4, 5])
def test_rmat12(schedule, rmat12):
    n, s, d = rmat12
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    print("case decompose rmat-s12-ef8 schedule=%d" % schedule, flush=True)
    want, want_k = oracle_trussness(rp, col)
    got, got_k = run(rp, col, schedule)
    assert got_k == want_k and np.array_equal(got, want)


@pytest.mark.parametrize("seed", [21, 22])
def test_rmat13_skewed_with_clique(seed):
    n, s, d = synth.rmat(13, 8, 0.6, 0.15, 0.15, seed)
    v = synth.distinct_vertices(n, 30, seed + 100)
    cs, cd = synth.clique_pairs(v)
    s, d = np.concatenate([s, cs]), np.concatenate([d, cd])
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    print("case decompose rmat-s13+clique30 seed=%d m=%d" % (seed, len(col)), flush=True)
    want, want_k = oracle_trussness(rp, col)
    assert want_k >= 30
    for schedule in (1, 4):
        got, got_k = run(rp, col, schedule)
        assert got_k == want_k and np.array_equal(got, want), schedule
