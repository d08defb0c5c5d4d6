"""The allocation-free entry point (ktruss_run_noalloc) through the C-ABI:
its masks, supports and pass counts equal ktruss_run's on the same graph,
for two calls in a row on the one fixed scratch array, the second on a
smaller graph (so that stale contents of the first call are in the array),
and under several schedules; sizes beyond the array are rejected."""
import ctypes

import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def noalloc(rp, col, schedule, K):
    import torch
    lib = kt().load()
    rp_d = torch.from_numpy(np.ascontiguousarray(rp, np.int32)).cuda()
    col_d = torch.from_numpy(np.ascontiguousarray(col if len(col) else np.zeros(1), np.int32)).cuda()
    m = len(col)
    mask = torch.empty(max(m, 1), dtype=torch.uint8, device="cuda")
    sup = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    rounds = ctypes.c_int32()
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.ktruss_run_noalloc(len(rp) - 1, m, rp_d.data_ptr(), col_d.data_ptr(), schedule, K, mask.data_ptr(),
                                sup.data_ptr(), ctypes.byref(rounds), ctypes.c_void_p(stream))
    assert rc == 0, lib.ktruss_last_error_message().decode()
    return mask[:m].cpu().numpy(), sup[:m].cpu().numpy(), rounds.value


def reference(rp, col, schedule, K):
    import torch
    g = kt().Graph(rp, col, device="cuda")
    kt().ktruss_set_schedule(g, schedule)
    mask, sup, rounds = kt().ktruss_run(g, K)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), sup.cpu().numpy(), rounds


def graphs():
    big = synth.workload_pairs("rmat-s12-ef8")
    n, s, d = synth.rmat(11, 8, 0.6, 0.15, 0.15, 9)
    return [("rmat-s12-ef8", big), ("rmat-s11-ef8", (n, s, d)), ("K8", synth.complete(8))]


@pytest.mark.parametrize("schedule", [0, 1, 4])
def test_two_calls_match_ktruss_run(schedule):
    for name, (n, s, d) in graphs():  # largest first: later calls find its contents in the array
        rp, col, _ = kt().ktruss_build_csr(s, d, n)
        for K in (3, 5):
            print("case noalloc %s m=%d schedule=%d K=%d" % (name, len(col), schedule, K), flush=True)
            got = noalloc(rp, col, schedule, K)
            want = reference(rp, col, schedule, K)
            assert got[2] == want[2]
            assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_rejects_sizes_beyond_the_scratch():
    lib = kt().load()
    rounds = ctypes.c_int32()
    # 50M edges need far more than the fixed array: refused before any device work
    rc = lib.ktruss_run_noalloc(1 << 20, 50_000_000, None, None, 0, 3, None, None, ctypes.byref(rounds), None)
    assert rc == kt().E_CAPACITY
    assert b"scratch" in lib.ktruss_last_error_message()
    rc = lib.ktruss_run_noalloc(10, 5, None, None, 2, 3, None, None, ctypes.byref(rounds), None)
    assert rc == kt().E_INVALID
