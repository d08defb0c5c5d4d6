"""Cost model on the GPU: the library's FP32 forward, gradient and Adam kernels
against the float64 reference (oracle/mlp.py, itself pinned by finite
differences), the learned schedule's results against the oracle under any
weights (the model steers scheduling only), and training on the library's own
timing samples."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available
from oracle import mlp as ref

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def kt():
    from paper_2009_07929_amd import ktruss
    return ktruss


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def data(seed, rows):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, ref.N_PARAMS)
    X = rng.normal(0, 1, (rows, 5))
    T = rng.normal(0, 1, rows)
    return theta, X, T


@pytest.mark.parametrize("rows", [1, 63, 64, 1000, 70000])
def test_forward_matches_reference(rows):
    theta, X, _ = data(rows, rows)
    theta32, X32 = theta.astype(np.float32), X.astype(np.float32)
    y = kt().ktruss_mlp_forward(dev(theta32), dev(X32)).cpu().numpy()
    want = ref.forward(theta32.astype(np.float64), X32.astype(np.float64))
    assert np.allclose(y, want, rtol=1e-4, atol=1e-4 * (1 + np.abs(want).max()))


@pytest.mark.parametrize("rows", [1, 64, 129, 5000, 100000])
def test_gradient_matches_reference(rows):
    theta, X, T = data(100 + rows, rows)
    theta32, X32, T32 = theta.astype(np.float32), X.astype(np.float32), T.astype(np.float32)
    loss, grad = kt().ktruss_mlp_loss_grad(dev(theta32), dev(X32), dev(T32))
    L, g = ref.loss_and_grad(theta32.astype(np.float64), X32.astype(np.float64), T32.astype(np.float64))
    grad = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - L) <= 1e-4 * abs(L)
    assert np.linalg.norm(grad - g) <= 1e-4 * np.linalg.norm(g)
    assert np.allclose(grad, g, rtol=1e-3, atol=1e-5 * np.abs(g).max())
    # deterministic reduction order
    _, grad2 = kt().ktruss_mlp_loss_grad(dev(theta32), dev(X32), dev(T32))
    assert np.array_equal(grad2.cpu().numpy(), grad.astype(np.float32))


def test_adam_matches_reference():
    import torch
    rng = np.random.default_rng(7)
    theta = rng.normal(0, 1, ref.N_PARAMS).astype(np.float32)
    m = np.zeros(ref.N_PARAMS, np.float32)
    v = np.zeros(ref.N_PARAMS, np.float32)
    p_d, m_d, v_d = dev(theta), dev(m), dev(v)
    th64, m64, v64 = theta.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 6):
        g = rng.normal(0, 1, ref.N_PARAMS).astype(np.float32)
        kt().ktruss_mlp_adam(p_d, dev(g), m_d, v_d, step, lr=0.01)
        th64, m64, v64 = ref.adam_step(th64, g.astype(np.float64), m64, v64, step, lr=0.01)
    torch.cuda.synchronize()
    assert np.allclose(p_d.cpu().numpy(), th64, rtol=1e-5, atol=1e-5)
    assert np.allclose(m_d.cpu().numpy(), m64, rtol=1e-4, atol=1e-6)


def learned_run(rp, col, K, params, tuning=None):
    import torch
    g = kt().Graph(rp, col, device="cuda")
    if tuning is None:
        tuning = kt().ktruss_tuning()
    tuning.plain_max_work = -1   # exercise the learned bins even on light graphs
    kt().ktruss_set_schedule(g, kt().SCHED_LEARNED, params, tuning)
    mask, sup, rounds = kt().ktruss_run(g, K)
    torch.cuda.synchronize()
    return mask.cpu().numpy(), sup.cpu().numpy(), rounds


@pytest.mark.parametrize("kind", ["random", "all-hub", "no-hub", "nan", "tiny-chunks"])
def test_learned_schedule_never_changes_results(kind, rmat12):
    n, s, d = rmat12
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    rng = np.random.default_rng(11)
    theta = rng.normal(0, 0.5, ref.N_PARAMS).astype(np.float32)
    t = kt().ktruss_tuning()
    if kind == "all-hub":
        theta[:] = 0
        theta[-1] = -40.0           # hub predicted 2^40 times cheaper everywhere: every row is a hub row
    elif kind == "no-hub":
        theta[:] = 0
        theta[-1] = 40.0            # nothing is a hub row: all tasks on wave/thread kernels
    elif kind == "nan":
        theta[:] = np.nan
    elif kind == "tiny-chunks":
        theta[-1] = -1.0
        t.hub_chunk_tasks = 16
        t.learned_hub_min = 0.5
    params = dev(theta)
    for K in (3, 4, 6, 9):
        print("case learned %s K=%d" % (kind, K), flush=True)
        gm, gs, gr = learned_run(rp, col, K, params, t)
        om, osup, orounds = oracle.truss(rp, col, K, "P")
        assert np.array_equal(gm, om) and np.array_equal(gs, osup) and gr == orounds


def test_learned_schedule_skewed_graph():
    n, s, d = synth.rmat(15, 16, 0.65, 0.15, 0.15, 71)
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    theta = np.random.default_rng(3).normal(0, 0.5, ref.N_PARAMS).astype(np.float32)
    theta[-1] = 0.0                 # a mix of hub and per-edge rows
    for K in (3, 7):
        gm, gs, gr = learned_run(rp, col, K, dev(theta))
        om, osup, orounds = oracle.truss(rp, col, K, "P")
        assert np.array_equal(gm, om) and np.array_equal(gs, osup) and gr == orounds


def test_cost_samples_and_training_beat_constant():
    import torch
    from paper_2009_07929_amd import cost_model
    graphs = [(13, 0.5, 1), (14, 0.6, 2), (15, 0.57, 3)]
    X, Y = cost_model.collect(graphs, Ks=(3, 5, 8), per_run_cap=200_000, log=lambda *a: None)
    assert X.shape[0] > 1000 and X.shape[1] == 5
    assert torch.isfinite(X).all() and torch.isfinite(Y).all()
    params, hist = cost_model.train(X, Y, steps=600, batch=8192, lr=3e-3, log=lambda *a: None, eval_every=300)
    step, train_mse, val_mse, const_mse, sign = hist[-1]
    print("cost model: held-out mse %.4f vs constant predictor %.4f, sign agreement %.3f"
          % (val_mse, const_mse, sign), flush=True)
    assert val_mse < 0.8 * const_mse


def test_trained_model_gains_on_measured_costs():
    """On a graph outside the training set, the per-row costs measured on both
    kernels (paired samples) are summed under three policies: every row on the
    hub kernel, every row on the wavefront kernel, and the trained network's
    choice (hub where it predicts the hub kernel cheaper).  The network's
    choice must cost less than either fixed policy; the gain is printed."""
    import torch
    from paper_2009_07929_amd import cost_model
    params = cost_model.load_params("cuda")
    assert params is not None, "the trained cost-model weights ship with the package"
    n, s, d = synth.rmat(17, 16, 0.62, 0.165, 0.165, 909)
    rp, col, _ = kt().ktruss_build_csr(s, d, n)
    g = kt().Graph(rp, col, device="cuda")
    Xh, Yh = kt().ktruss_collect_row_costs(g, 5, 2_000_000, variant=cost_model.HUB)
    Xw, Yw = kt().ktruss_collect_row_costs(g, 5, 2_000_000, variant=cost_model.WAVE)
    assert len(Yh) == len(Yw) and torch.equal(Xh, Xw)
    hub = torch.exp2(Yh.double()) - 1
    wave = torch.exp2(Yw.double()) - 1
    pred = kt().ktruss_mlp_forward(params, Xh)
    choice = torch.where(pred <= 0, hub, wave)
    c_hub, c_wave, c_net, c_best = (float(v.sum()) for v in (hub, wave, choice, torch.minimum(hub, wave)))
    print("measured wave-cycles: all hub %.3e, all wavefront %.3e, network %.3e (best per row %.3e); "
          "gain %.3fx over all-hub, %.3fx over all-wavefront" % (c_hub, c_wave, c_net, c_best, c_hub / c_net,
                                                                 c_wave / c_net), flush=True)
    assert c_net < c_hub and c_net < c_wave
