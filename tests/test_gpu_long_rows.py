"""Rows long enough for the per-row hit-word sum (k_hit_sum_long: rows of
193 to 4,096 edges) and for its neighbours on both sides of those bounds,
under the hub and heuristic schedules, recomputing and with incremental
maintenance.

Pins that do not need the oracle: in the complete graph K_n every edge lies in
n - 2 triangles, so for K <= n the K-truss is the whole graph with supports
n - 2 after one pass that removes nothing, and for K = n + 1 the first pass
removes every edge and a second finds nothing left.  The mixed graph (R-MAT
plus planted cliques of 150, 260 and 450 vertices, so that rows of every
length class meet in one run) is compared with the oracle bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def run(rp, col, K, schedule, incremental):
    import torch
    g = kt().Graph(rp, col, device="cuda")
    t = kt().ktruss_tuning()
    t.plain_max_work = -1
    t.incremental = incremental
    kt().ktruss_set_schedule(g, schedule, None, t)
    mask, sup, rounds = kt().ktruss_run(g, K)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), sup.cpu().numpy(), rounds


@pytest.mark.parametrize("n", [190, 194, 300, 1100])
@pytest.mark.parametrize("schedule", [1, 4])
def test_complete_graph_closed_form(n, schedule):
    rp, col, _ = kt().ktruss_build_csr(*synth.complete(n)[1:], n)
    m = n * (n - 1) // 2
    assert len(col) == m
    for K in (3, n, n + 1):
        for inc in (0, 2):
            print("case K_%d K=%d schedule=%d incremental=%d" % (n, K, schedule, inc), flush=True)
            mask, sup, rounds = run(rp, col, K, schedule, inc)
            if K <= n:
                assert mask.all() and (sup == n - 2).all(), (n, K)
                assert rounds == 1
            else:
                assert not mask.any() and not sup.any(), (n, K)
                assert rounds == 2


def mixed_graph():
    n, s, d = synth.rmat(14, 8, 0.57, 0.19, 0.19, 41)
    parts_s, parts_d = [s], [d]
    for size, seed in ((150, 401), (260, 402), (450, 403)):
        cs, cd = synth.clique_pairs(synth.distinct_vertices(n, size, seed))
        parts_s.append(cs)
        parts_d.append(cd)
    return n, np.concatenate(parts_s), np.concatenate(parts_d)


MIXED = mixed_graph()
_ORACLE = {}


def oracle_truss(rp, col, K):
    if K not in _ORACLE:
        _ORACLE[K] = oracle.truss(rp, col, K, "P")
    return _ORACLE[K]


@pytest.mark.parametrize("schedule", [1, 4])
@pytest.mark.parametrize("incremental", [0, 2])
def test_mixed_row_lengths_match_oracle(schedule, incremental):
    n, s, d = MIXED
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    lengths = np.diff(rp)
    # rows on both sides of the per-row bounds are present
    assert (lengths > 192).sum() > 0 and ((lengths > 64) & (lengths <= 192)).sum() > 0
    for K in (3, 8, 40, 150, 260, 450):
        print("case mixed m=%d K=%d schedule=%d incremental=%d" % (len(col), K, schedule, incremental), flush=True)
        mask, sup, rounds = run(rp, col, K, schedule, incremental)
        om, osup, orounds = oracle_truss(rp, col, K)
        assert rounds == orounds, (K, rounds, orounds)
        assert np.array_equal(mask, om), K
        assert np.array_equal(sup, osup), K
