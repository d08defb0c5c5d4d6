"""Training of the learned scheduler's cost model.

Samples come from the library itself (ktruss_collect_row_costs): the same
fixpoint run twice, once with every task on the workgroup-per-hub-row kernel
and once on the wavefront-per-edge kernel, each timed per row with the shader
clock in wave-cycles; both runs visit the same rows in the same order, so each
(row, pass) sample pairs the two costs with the five row features the
LEARNED schedule computes.  The target is log2(hub cost) - log2(wavefront
cost): the schedule sends a row to the hub kernel when the prediction is at
most its threshold.  Training runs on the GPU with the library's own gradient
and Adam kernels.  The trained parameters (4,609 float32) steer scheduling
only.
"""
from __future__ import annotations

import os

import numpy as np

from . import ktruss as kt

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "cost_model_weights.npy")

# Training graphs: R-MAT scales 14-20 with varied quadrant probabilities
# (a from 0.45 to 0.70, b = c, d >= 0.05), K in 3..12.
TRAIN_GRAPHS = [(14, 0.45, 100), (15, 0.55, 101), (16, 0.65, 102), (17, 0.50, 103), (18, 0.60, 104),
                (19, 0.57, 105), (20, 0.70, 106), (18, 0.45, 107), (20, 0.52, 108)]
TRAIN_KS = (3, 4, 5, 6, 8, 10, 12)
HUB, WAVE = 0, 1


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation (float32), drawn on the host and passed to the GPU."""
    rng = np.random.default_rng(seed)
    h, i = kt.MLP_HIDDEN, kt.MLP_IN
    parts = [rng.normal(0, np.sqrt(2.0 / i), h * i), np.zeros(h), rng.normal(0, np.sqrt(2.0 / h), h * h),
             np.zeros(h), rng.normal(0, np.sqrt(1.0 / h), h), np.array([0.0])]
    return np.concatenate(parts).astype(np.float32)


def paired_samples(g, K, cap):
    """(X, log2 hub cost - log2 wavefront cost) of one run; the two timed runs
    must list the same rows with the same features."""
    import torch
    Xh, Yh = kt.ktruss_collect_row_costs(g, K, cap, variant=HUB)
    Xw, Yw = kt.ktruss_collect_row_costs(g, K, cap, variant=WAVE)
    n = min(len(Yh), len(Yw))
    if len(Yh) != len(Yw) or not torch.equal(Xh[:n], Xw[:n]):
        raise RuntimeError("hub and wavefront samples do not pair up")
    return Xh[:n].clone(), (Yh[:n] - Yw[:n]).clone()


def collect(graphs=TRAIN_GRAPHS, Ks=TRAIN_KS, per_run_cap=400_000, device="cuda", log=print):
    """(X[N,5], Y[N]) device tensors of paired per-row cost samples."""
    import torch
    import synth
    xs, ys = [], []
    for scale, a, seed in graphs:
        bc = (1.0 - a - 0.05) / 2.0
        n, s, d = synth.rmat(scale, 16, a, bc, bc, seed)
        rp, col, _ = kt.ktruss_build_csr(s, d, n)
        g = kt.Graph(rp, col, device=device)
        for K in Ks:
            X, Y = paired_samples(g, K, per_run_cap)
            xs.append(X)
            ys.append(Y)
        torch.cuda.synchronize()
        log("samples: R-MAT scale %d a=%.2f: %d so far" % (scale, a, sum(len(y) for y in ys)))
        del g
    return torch.cat(xs), torch.cat(ys)


def train(X, Y, steps=3000, batch=65536, lr=2e-3, seed=0, log=print, eval_every=500):
    """Adam on mini-batches of a one-time shuffle.  Returns (params tensor, history)."""
    import torch
    n = X.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(n, generator=gen).to(X.device)
    Xs, Ys = X[perm].contiguous(), Y[perm].contiguous()
    n_val = max(1, n // 10)
    Xv, Yv = Xs[:n_val].contiguous(), Ys[:n_val].contiguous()
    Xt, Yt = Xs[n_val:].contiguous(), Ys[n_val:].contiguous()
    params = torch.from_numpy(init_params(seed)).to(X.device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    nt = Xt.shape[0]
    hist = []
    work = None
    for step in range(1, steps + 1):
        lo = ((step - 1) * batch) % max(nt - batch, 1)
        xb, yb = Xt[lo:lo + batch], Yt[lo:lo + batch]
        loss, grad = kt.ktruss_mlp_loss_grad(params, xb, yb, work)
        kt.ktruss_mlp_adam(params, grad, m, v, step, lr=lr)
        if step % eval_every == 0 or step == steps:
            vl, _ = kt.ktruss_mlp_loss_grad(params, Xv, Yv)
            const = float(((Yv - Yt.mean()) ** 2).mean().item())
            pv = kt.ktruss_mlp_forward(params, Xv)
            sign = float(((pv <= 0) == (Yv <= 0)).float().mean().item())
            hist.append((step, float(loss.item()), float(vl.item()), const, sign))
            log("step %d train mse %.4f  held-out mse %.4f  (constant predictor %.4f)  held-out sign agreement %.3f"
                % hist[-1])
    return params, hist


def load_params(device="cuda"):
    """The committed trained parameters as a device tensor (None if absent)."""
    import torch
    if not os.path.exists(WEIGHTS):
        return None
    return torch.from_numpy(np.load(WEIGHTS).astype(np.float32)).to(device)


if __name__ == "__main__":
    # python -m paper_2009_07929_amd.cost_model [output directory (default: the package)]
    import json
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    out_dir = sys.argv[1] if len(sys.argv) > 1 else HERE
    X, Y = collect()
    params, hist = train(X, Y, steps=int(os.environ.get("COST_MODEL_STEPS", "4000")))
    np.save(os.path.join(out_dir, "cost_model_weights.npy"), params.cpu().numpy())
    with open(os.path.join(out_dir, "cost_model_train.json"), "w") as f:
        json.dump({"samples": int(X.shape[0]), "target": "log2 hub wave-cycles - log2 wavefront wave-cycles",
                   "graphs": TRAIN_GRAPHS, "Ks": TRAIN_KS, "history": hist}, f, indent=1)
    print("saved to", out_dir, "samples", X.shape[0], "final", hist[-1])
