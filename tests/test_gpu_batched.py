"""Batched form and hipGraph-replayed rounds: results must equal separate
per-graph runs and the oracle, bit for bit, under every schedule."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

SCHEDULES = [0, 1, 3, 4, 5]  # plain, heuristic, force-wave, force-hub, coarse


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def mixed_graphs(count, seed):
    """Small graphs of uneven sizes: Chung-Lu, R-MAT, cliques, paths, empty."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(count):
        kind = g % 6
        if kind == 0:
            n, s, d = synth.chung_lu(int(rng.integers(64, 600)), float(rng.uniform(2.1, 3.0)),
                                     float(rng.uniform(4, 32)), 1000 + g)
        elif kind == 1:
            n, s, d = synth.rmat(int(rng.integers(7, 10)), 8, 0.6, 0.15, 0.15, 2000 + g)
        elif kind == 2:
            n, s, d = synth.complete(int(rng.integers(3, 12)))
        elif kind == 3:
            n, s, d = synth.path(int(rng.integers(2, 30)))
        elif kind == 4:
            n, s, d = int(rng.integers(1, 20)), np.zeros(0, np.int32), np.zeros(0, np.int32)
        else:
            n, s, d = synth.erdos_renyi(int(rng.integers(10, 80)), float(rng.uniform(0.05, 0.4)), 3000 + g)
        rp, col, _ = kt().ktruss_build_csr(s, d, n)
        out.append((rp, col))
    K = rng.integers(3, 9, size=count).astype(np.int32)
    return out, K


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_batched_equals_oracle(schedule):
    import torch
    graphs, K = mixed_graphs(60, 7)
    b = kt().Batch(graphs, device="cuda", schedule=schedule)
    print("case batched G=%d m_total=%d schedule=%d" % (b.G, b.m_total, schedule), flush=True)
    mask, sup, rounds = kt().ktruss_run_batched(b, K)
    torch.cuda.synchronize()
    mask, sup, rounds = mask.cpu().numpy(), sup.cpu().numpy(), rounds.cpu().numpy()
    eo = b.edge_offsets()
    for g, (rp, col) in enumerate(graphs):
        om, osup, orounds = oracle.truss(rp, col, int(K[g]), "P")
        assert np.array_equal(mask[eo[g]:eo[g + 1]], om), g
        assert np.array_equal(sup[eo[g]:eo[g + 1]], osup), g
        assert rounds[g] == orounds, (g, rounds[g], orounds)


def test_batched_equals_single_runs():
    import torch
    graphs, K = mixed_graphs(24, 11)
    b = kt().Batch(graphs, device="cuda", schedule=1)
    mask, sup, rounds = kt().ktruss_run_batched(b, K)
    torch.cuda.synchronize()
    eo = b.edge_offsets()
    for g, (rp, col) in enumerate(graphs):
        gr = kt().Graph(rp, col, device="cuda", schedule=1)
        m1, s1, r1 = kt().ktruss_run(gr, int(K[g]))
        torch.cuda.synchronize()
        assert np.array_equal(mask.cpu().numpy()[eo[g]:eo[g + 1]], m1.cpu().numpy())
        assert np.array_equal(sup.cpu().numpy()[eo[g]:eo[g + 1]], s1.cpu().numpy())
        assert int(rounds[g].item()) == r1


@pytest.mark.parametrize("rps", [2, 3, 8])
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_graph_replay_equals_host_loop(rps, schedule, rmat12):
    import torch
    n, s, d = rmat12
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    g = kt().Graph(rp, col, device="cuda", schedule=schedule)
    t = kt().ktruss_tuning()
    t.rounds_per_sync = rps
    t.plain_max_work = -1
    kt().ktruss_set_schedule(g, schedule, None, t)
    for K in (3, 5, 8, 30):
        print("case graph-replay rps=%d schedule=%d K=%d" % (rps, schedule, K), flush=True)
        mask, sup, rounds = kt().ktruss_run(g, K)
        torch.cuda.synchronize()
        om, osup, orounds = oracle.truss(rp, col, K, "P")
        assert np.array_equal(mask.cpu().numpy(), om)
        assert np.array_equal(sup.cpu().numpy(), osup)
        assert rounds == orounds


def test_batched_graph_replay():
    import torch
    graphs, K = mixed_graphs(30, 5)
    b = kt().Batch(graphs, device="cuda", schedule=1)
    t = kt().ktruss_tuning()
    t.rounds_per_sync = 4
    b.c.tuning = t
    mask, sup, rounds = kt().ktruss_run_batched(b, K)
    torch.cuda.synchronize()
    eo = b.edge_offsets()
    for g, (rp, col) in enumerate(graphs):
        om, osup, orounds = oracle.truss(rp, col, int(K[g]), "P")
        assert np.array_equal(mask.cpu().numpy()[eo[g]:eo[g + 1]], om)
        assert np.array_equal(sup.cpu().numpy()[eo[g]:eo[g + 1]], osup)
        assert int(rounds[g].item()) == orounds


def test_batched_rejects_malformed():
    graphs, K = mixed_graphs(6, 3)
    vert_off, rowptr, col = kt().union_csr(graphs)
    # an edge from graph 0 into graph 1
    bad_col = col.copy()
    r0 = int(np.flatnonzero(np.diff(rowptr[: vert_off[1] + 1]))[0])   # a non-empty row of graph 0
    e = int(rowptr[r0 + 1]) - 1
    bad_col[e] = vert_off[1] + 1
    if rowptr[r0 + 1] - rowptr[r0] > 1:
        pass
    b = kt().Batch(None, device="cuda", vert_off=vert_off, rowptr=rowptr, col=bad_col)
    print("case batched crossing edge", flush=True)
    with pytest.raises(kt().KtrussError) as ei:
        kt().ktruss_run_batched(b, K)
    assert ei.value.code == kt().E_INVALID
    b = kt().Batch(graphs, device="cuda")
    K2 = K.copy()
    K2[2] = 1
    print("case batched K<2", flush=True)
    with pytest.raises(kt().KtrussError) as ei:
        kt().ktruss_run_batched(b, K2)
    assert ei.value.code == kt().E_INVALID


def test_autotuner_picks_a_bit_exact_config(tmp_path, rmat12):
    import torch
    from paper_2009_07929_amd import autotune
    n, s, d = rmat12
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    g = kt().Graph(rp, col, device="cuda")
    path = str(tmp_path / "cache.json")
    key, best, t = autotune.tune_graph(g, 5, reps=1, path=path, rowptr=rp)
    assert autotune.tuned_config(key, path) == best and t > 0
    mask, sup, rounds = kt().ktruss_run(g, 5)
    torch.cuda.synchronize()
    om, osup, orounds = oracle.truss(rp, col, 5, "P")
    assert np.array_equal(mask.cpu().numpy(), om) and np.array_equal(sup.cpu().numpy(), osup) and rounds == orounds
    graphs, K = mixed_graphs(20, 9)
    b = kt().Batch(graphs, device="cuda")
    key, best, t = autotune.tune_batch(b, torch.from_numpy(K).cuda(), reps=1, path=path)
    print("case autotuned batch config %s" % best, flush=True)
    mask, sup, rounds = kt().ktruss_run_batched(b, K)
    torch.cuda.synchronize()
    eo = b.edge_offsets()
    for gi, (rp2, col2) in enumerate(graphs):
        om, osup, orounds = oracle.truss(rp2, col2, int(K[gi]), "P")
        assert np.array_equal(mask.cpu().numpy()[eo[gi]:eo[gi + 1]], om)
        assert int(rounds[gi].item()) == orounds
