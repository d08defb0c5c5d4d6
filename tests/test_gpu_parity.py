"""GPU parity: the HIP path through the C-ABI against the CPU oracle, bit for bit
(all of this is integer work: masks, supports and round counts must be equal)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def build(g, order=1):
    n, s, d = g
    rp, col, n2o = kt().ktruss_build_csr(s, d, n, order)
    return rp, col, n2o


def run_gpu(rp, col, K, schedule=0):
    import torch
    g = kt().Graph(rp, col, device="cuda")
    if schedule:
        t = kt().ktruss_tuning()
        t.plain_max_work = -1   # exercise the schedule even on light graphs
        kt().ktruss_set_schedule(g, schedule, None, t)
    mask, sup, rounds = kt().ktruss_run(g, K)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), sup.cpu().numpy(), rounds


def assert_parity(rp, col, K, schedule=0, label=""):
    print("case %s K=%d m=%d schedule=%d" % (label, K, len(col), schedule), flush=True)
    gm, gs, gr = run_gpu(rp, col, K, schedule)
    om, osup, orounds = oracle.truss(rp, col, K, "P")
    assert np.array_equal(gm, om), (label, K, "mask")
    assert np.array_equal(gs, osup), (label, K, "support")
    assert gr == orounds, (label, K, gr, orounds)


SMALL = {
    "K3": synth.complete(3), "K5": synth.complete(5), "K9": synth.complete(9),
    "path": synth.path(10), "star": synth.star(12), "C8": synth.cycle(8), "K34": synth.complete_bipartite(3, 4),
    "petersen": synth.petersen(), "grid": synth.grid(5, 6), "er": synth.erdos_renyi(60, 0.3, 4),
    "empty": (6, np.zeros(0, np.int32), np.zeros(0, np.int32)), "one-edge": (3, np.array([0], np.int32), np.array([2], np.int32)),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_small_graphs(name):
    rp, col, _ = build(SMALL[name])
    for K in (2, 3, 4, 5, 7, 10):
        assert_parity(rp, col, K, label=name)


SCHEDULES = [0, 1, 3, 4, 5]   # plain, heuristic, force-wave, force-hub, coarse (thread per row)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("K", [2, 3, 4, 5, 6, 8, 12, 20, 100])
def test_rmat12(K, schedule, rmat12):
    rp, col, _ = build(rmat12)
    assert_parity(rp, col, K, schedule, label="rmat-s12-ef8")


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("name", sorted(SMALL))
def test_small_graphs_schedules(name, schedule):
    rp, col, _ = build(SMALL[name])
    for K in (3, 4, 6):
        assert_parity(rp, col, K, schedule, label=name)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("seed", [0, 1])
def test_rmat14_skewed(seed, schedule):
    rp, col, _ = build(synth.rmat(14, 16, 0.65, 0.15, 0.15, 40 + seed))
    for K in (3, 5, 9, 16):
        assert_parity(rp, col, K, schedule, label="rmat-s14-ef16-skew%d" % seed)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_wide_rows_and_spans(schedule):
    # order=0 keeps ids: rows get long (beyond the LDS key capacity) and label
    # spans get wide (beyond the bitmap span), exercising the sorted-key and
    # global-memory lookups of the hub kernel.
    n, s, d = synth.rmat(15, 16, 0.6, 0.15, 0.15, 91)
    rp, col, _ = build((n, s, d), order=2)
    for K in (3, 6):
        assert_parity(rp, col, K, schedule, label="rmat-s15 descending order")
    rp, col, _ = build((n, s, d), order=0)
    for K in (3, 6):
        assert_parity(rp, col, K, schedule, label="rmat-s15 natural order")


@pytest.mark.parametrize("order", [0, 2])
def test_other_orders(order, rmat12):
    rp, col, _ = build(rmat12, order)
    for K in (3, 6):
        assert_parity(rp, col, K, label="rmat-s12 order=%d" % order)


def test_planted_clique():
    n, s, d = synth.rmat(13, 8, 0.6, 0.15, 0.15, 77)
    cs, cd = synth.clique_pairs(synth.distinct_vertices(n, 64, 78))
    rp, col, _ = build((n, np.concatenate([s, cs]), np.concatenate([d, cd])))
    for K in (3, 20, 64, 65):
        for schedule in SCHEDULES:
            assert_parity(rp, col, K, schedule, label="rmat13+clique64")


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_support_and_prune_calls(schedule, rmat12):
    import torch
    rp, col, _ = build(rmat12)
    g = kt().Graph(rp, col, device="cuda")
    kt().ktruss_set_schedule(g, schedule)
    print("case ktruss_support all-alive", flush=True)
    sup = kt().ktruss_support(g).cpu().numpy()
    assert np.array_equal(sup, oracle.supports(rp, col))
    rng = np.random.default_rng(5)
    alive = (rng.random(len(col)) < 0.7).astype(np.uint8)
    alive_d = torch.from_numpy(alive).cuda()
    print("case ktruss_support random alive", flush=True)
    sup = kt().ktruss_support(g, alive_d).cpu().numpy()
    assert np.array_equal(sup, oracle.supports(rp, col, alive))
    print("case ktruss_prune", flush=True)
    removed = torch.zeros(1, dtype=torch.int64, device="cuda")
    sup_d = torch.from_numpy(sup).cuda()
    kt().ktruss_prune(g, 5, sup_d, alive_d, removed)
    want, nrem = oracle.prune(sup, alive, 5)
    assert np.array_equal(alive_d.cpu().numpy(), want) and int(removed.item()) == nrem


@pytest.mark.parametrize("K", [4, 7])
def test_iterated_steps_equal_run(K, rmat12):
    import torch
    rp, col, _ = build(rmat12)
    g = kt().Graph(rp, col, device="cuda")
    alive = torch.ones(len(col), dtype=torch.uint8, device="cuda")
    removed = torch.zeros(1, dtype=torch.int64, device="cuda")
    passes = 0
    print("case iterated support/prune K=%d" % K, flush=True)
    while True:
        sup = kt().ktruss_support(g, alive)
        passes += 1
        kt().ktruss_prune(g, K, sup, alive, removed)
        if int(removed.item()) == 0:
            break
    mask, rsup, rounds = kt().ktruss_run(g, K)
    assert np.array_equal(alive.cpu().numpy(), mask.cpu().numpy())
    assert np.array_equal(sup.cpu().numpy(), rsup.cpu().numpy())
    assert passes == rounds


def test_repeat_runs_identical(rmat12):
    rp, col, _ = build(rmat12)
    a = run_gpu(rp, col, 5)
    for _ in range(3):
        b = run_gpu(rp, col, 5)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_malformed_csr_rejected():
    import torch
    ok_rp = np.array([0, 2, 3, 3], np.int32)
    ok_col = np.array([1, 2, 2], np.int32)
    cases = {
        "descending": (ok_rp, np.array([2, 1, 2], np.int32)),
        "below-diagonal": (ok_rp, np.array([1, 2, 1], np.int32)),
        "col>=n": (ok_rp, np.array([1, 2, 3], np.int32)),
        "rowptr-end": (np.array([0, 2, 3, 2], np.int32), ok_col),
        "rowptr-start": (np.array([1, 2, 3, 3], np.int32), ok_col),
    }
    for name, (rp, col) in cases.items():
        print("case malformed %s" % name, flush=True)
        g = kt().Graph(rp, col, device="cuda")
        with pytest.raises(kt().KtrussError) as ei:
            kt().ktruss_run(g, 3)
        assert ei.value.code == kt().E_INVALID, name
    torch.cuda.synchronize()
