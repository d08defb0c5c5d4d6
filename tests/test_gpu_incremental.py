"""Incremental support maintenance (tuning.incremental = 1 or 2) against the
oracle: after the first pass the survivors keep their supports and each prune
takes off the triangles it destroys, charged once.  Mask, supports and the
pass count must equal the recompute loop's (oracle mode P, whose peel is the
CPU form of the same rule) bit for bit, under every schedule, with
host-checked and graph-replayed rounds, for the auto mode at several ratios
(so that peeled and recomputed rounds mix), and in the truss decomposition."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def graphs():
    out = [("K9", synth.complete(9)), ("petersen", synth.petersen()),
           ("two-K6", synth.disjoint_union(synth.complete(6), synth.complete(6))),
           ("er-120", synth.erdos_renyi(120, 0.2, 5)),
           ("rmat-s12-ef8", synth.workload_pairs("rmat-s12-ef8"))]
    n, s, d = synth.rmat(13, 8, 0.6, 0.15, 0.15, 31)
    cs, cd = synth.clique_pairs(synth.distinct_vertices(n, 40, 131))
    out.append(("rmat-s13+clique40", (n, np.concatenate([s, cs]), np.concatenate([d, cd]))))
    out.append(("chunglu-6000", synth.chung_lu(6000, 2.3, 24.0, 77)))
    out.append(("ba-5000", synth.barabasi_albert(5000, 6, 78)))
    return out


GRAPHS = graphs()


def run(rp, col, K, schedule, incremental, ratio=0, rps=0):
    import torch
    g = kt().Graph(rp, col, device="cuda")
    t = kt().ktruss_tuning()
    t.plain_max_work = -1
    t.rounds_per_sync = rps
    t.incremental = incremental
    t.peel_ratio = ratio
    kt().ktruss_set_schedule(g, schedule, None, t)
    mask, sup, rounds = kt().ktruss_run(g, K)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), sup.cpu().numpy(), rounds


@pytest.mark.parametrize("idx", range(len(GRAPHS)))
def test_incremental_matches_oracle(idx):
    name, (n, s, d) = GRAPHS[idx]
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    for K in (2, 3, 4, 6, 9, 14, 1000):  # 2: nothing can go; 1000: everything goes
        om, osup, orounds = oracle.truss(rp, col, K, "P")
        for sched in (0, 1, 4, 5):
            for inc, ratio, rps in ((1, 0, 0), (2, 1, 0), (2, 4, 0), (2, 0.25, 0), (1, 0, 3), (2, 0.25, 4)):
                print("case incremental %s m=%d K=%d schedule=%d mode=%d ratio=%g rps=%d"
                      % (name, len(col), K, sched, inc, ratio, rps), flush=True)
                mask, sup, rounds = run(rp, col, K, sched, inc, ratio, rps)
                assert rounds == orounds, (K, sched, inc, rounds, orounds)
                assert np.array_equal(mask, om), (K, sched, inc)
                assert np.array_equal(sup, osup), (K, sched, inc)


def test_incremental_decomposition():
    import torch
    n, s, d = GRAPHS[5][1]
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    g = kt().Graph(rp, col, device="cuda")
    t = kt().ktruss_tuning()
    t.plain_max_work = -1
    want = None
    for inc in (0, 1, 2):
        t.incremental = inc
        kt().ktruss_set_schedule(g, 4, None, t)
        print("case incremental decomposition mode=%d" % inc, flush=True)
        tr, kmax = kt().ktruss_decompose(g)
        torch.cuda.synchronize()
        got = (tr.cpu().numpy(), kmax)
        if want is None:
            want = got
            assert kmax >= 40
        assert got[1] == want[1] and np.array_equal(got[0], want[0]), inc
    # against the oracle's levels
    levels = np.full(len(col), 2, np.int32)
    for K in range(3, want[1] + 2):
        mask, _, _ = oracle.truss(rp, col, K, "P")
        levels[mask.astype(bool)] = K
    assert np.array_equal(levels, want[0])


def test_incremental_rejects_bad_modes():
    n, s, d = synth.complete(5)
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    g = kt().Graph(rp, col, device="cuda")
    for inc, ratio in ((3, 0), (-1, 0), (2, -1.0), (2, float("nan"))):
        t = kt().ktruss_tuning()
        t.incremental = inc
        t.peel_ratio = ratio
        kt().ktruss_set_schedule(g, 0, None, t)
        with pytest.raises(kt().KtrussError):
            kt().ktruss_run(g, 3)


@pytest.mark.parametrize("seed,count", [(17, 60), (9, 20)])
@pytest.mark.parametrize("schedule", [0, 1, 4])
@pytest.mark.parametrize("inc,ratio,rps", [(0, 0, 4), (0, 0, 16), (1, 0, 0), (1, 0, 4), (1, 0, 16), (2, 1, 0),
                                           (2, 0.25, 0), (2, 4, 0), (2, 0.25, 16)])
def test_incremental_batched(schedule, inc, ratio, rps, seed, count):
    """The batched form with incremental maintenance (and, for reference,
    recomputing with graph-replayed rounds): graphs that finish leave the
    working set without destroying triangles; every graph's mask, supports
    and pass count equal the oracle's."""
    import torch
    from test_gpu_batched import mixed_graphs
    graphs, K = mixed_graphs(count, seed)
    b = kt().Batch(graphs, device="cuda", schedule=schedule)
    t = kt().ktruss_tuning()
    t.incremental = inc
    t.peel_ratio = ratio
    t.rounds_per_sync = rps
    b.c.tuning = t
    print("case incremental batched G=%d m_total=%d schedule=%d mode=%d ratio=%g rps=%d"
          % (b.G, b.m_total, schedule, inc, ratio, rps), flush=True)
    mask, sup, rounds = kt().ktruss_run_batched(b, K)
    torch.cuda.synchronize()
    mask, sup, rounds = mask.cpu().numpy(), sup.cpu().numpy(), rounds.cpu().numpy()
    eo = b.edge_offsets()
    bad = []
    for g, (rp, col) in enumerate(graphs):
        om, osup, orounds = oracle.truss(rp, col, int(K[g]), "P")
        if not (np.array_equal(mask[eo[g]:eo[g + 1]], om) and np.array_equal(sup[eo[g]:eo[g + 1]], osup)
                and rounds[g] == orounds):
            bad.append((g, int(K[g]), len(col), int(rounds[g]), orounds))
    assert not bad, bad
