"""Butterfly counting on the GPU (ktruss_butterflies) against the butterfly
oracle: per-edge counts and the total, exactly, on complete bipartite graphs
(closed forms), cycles and trees (none), seeded power-law bipartite graphs of
both orientations (so that either side becomes the pair side), graphs whose
pair vertices need the dense-window path (many wedges), and empty sides;
malformed inputs are rejected."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def gpu_count(nu, nv, rp, col):
    import torch
    cnt, total = kt().ktruss_butterflies(nu, nv, rp, col, device="cuda")
    torch.cuda.synchronize()
    return cnt.cpu().numpy(), total


def check(nu, nv, rp, col, name):
    print("case butterfly %s nu=%d nv=%d m=%d" % (name, nu, nv, len(col)), flush=True)
    want, want_total = oracle.butterflies(nu, nv, rp, col)
    got, total = gpu_count(nu, nv, rp, col)
    assert total == want_total, (name, total, want_total)
    assert np.array_equal(got, want), name
    return total


@pytest.mark.parametrize("a,b", [(1, 1), (2, 2), (3, 5), (7, 4), (40, 3), (3, 70)])
def test_complete_bipartite(a, b):
    n, s, d = synth.complete_bipartite(a, b)
    u, v = np.minimum(s, d), np.maximum(s, d) - a  # sides [0, a) and [a, a + b)
    rp, col = synth.bipartite_csr(a, b, u, v)
    total = check(a, b, rp, col, "K%d,%d" % (a, b))
    assert total == (a * (a - 1) // 2) * (b * (b - 1) // 2)


def test_even_cycle_and_star():
    # C8 as a bipartite graph: u_i - v_i - u_{i+1}; no 4-cycle
    k = 4
    u = np.array([i for i in range(k)] * 2, np.int32)
    v = np.array([i for i in range(k)] + [(i - 1) % k for i in range(k)], np.int32)
    rp, col = synth.bipartite_csr(k, k, u, v)
    assert check(k, k, rp, col, "C8") == 0
    rp, col = synth.bipartite_csr(1, 50, np.zeros(50, np.int32), np.arange(50, dtype=np.int32))
    assert check(1, 50, rp, col, "star") == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("shape", [(3000, 800, 2.4, 2.2, 25000), (600, 4000, 2.2, 2.6, 25000),
                                   (2000, 2000, 2.1, 2.1, 60000)])
def test_power_law(shape, seed):
    nu, nv, gu, gv, pairs = shape
    nu, nv, u, v = synth.bipartite_chung_lu(nu, nv, gu, gv, pairs, seed)
    rp, col = synth.bipartite_csr(nu, nv, u, v)
    check(nu, nv, rp, col, "chung-lu %s seed=%d" % (shape, seed))


def test_window_path():
    # a dense core: some pair vertices have far more wedges than the LDS hash takes
    nu, nv, u, v = synth.bipartite_chung_lu(20000, 600, 3.0, 2.05, 200000, 11)
    rp, col = synth.bipartite_csr(nu, nv, u, v)
    dv = np.bincount(col, minlength=nv)
    assert (dv * (dv - 1)).sum() > 0
    check(nu, nv, rp, col, "dense core")


def test_empty_sides():
    rp = np.zeros(6, np.int32)
    got, total = gpu_count(5, 0, rp, np.zeros(0, np.int32))
    assert total == 0 and len(got) == 0
    got, total = gpu_count(0, 7, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert total == 0


def test_malformed_rejected():
    rp = np.array([0, 2, 3], np.int32)
    with pytest.raises(kt().KtrussError):
        gpu_count(2, 3, rp, np.array([1, 0, 2], np.int32))   # columns not ascending
    with pytest.raises(kt().KtrussError):
        gpu_count(2, 3, rp, np.array([0, 1, 3], np.int32))   # column outside [0, nv)
    with pytest.raises(kt().KtrussError):
        gpu_count(2, 3, np.array([0, 3, 2], np.int32), np.array([0, 1, 2], np.int32))  # rowptr not monotone
