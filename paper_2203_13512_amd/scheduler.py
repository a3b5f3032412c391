"""Learned root scheduling: data collection, training and the saved model.

The model is the library's MLP (4 -> 64 -> 64 -> 1, ReLU, FP32), trained and
evaluated by its own HIP kernels (kc_mlp_train_step / kc_mlp_forward).  Its
inputs are the four per-root features that BitCol's staging records -- DAG
out-degree d+, core number, number of colors of G_u, edges of G_u -- as
log1p values standardised with the training set's mean and deviation; the
target is log1p of the root's listing work (BitJoins times words per
bitmap), which the listing kernels record per root.

The library uses the prediction to order roots (heaviest first) and to decide
how deep to split each root into queue items; the degree schedule, which
uses d+ alone, is the fallback.  Neither changes any count.

Run ``python -m paper_2203_13512_amd.scheduler`` on a GPU to collect the logs
of the training workloads, train, and write scheduler_mlp.json.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

import paper_2203_13512_amd as kc

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "scheduler_mlp.json")

# Training workloads: the generators of workloads 1-3, logged at the k of
# each model; 2 and 3 are shrunk so that logging them takes seconds.
# {k: [(workload, scale), ...]}
TRAIN_SETS = {
    7: [(1, 1.0), (2, 0.25), (3, 1 / 8)],
    8: [(1, 1.0), (2, 0.1), (3, 1 / 16)],
}


def load_model(device, k: int = 8, path: str = MODEL_PATH):
    """(params, norm) device tensors of the model trained for k (the nearest
    trained k otherwise), or None when no model has been saved."""
    if not os.path.exists(path):
        return None
    import torch
    with open(path) as f:
        models = json.load(f)["models"]
    key = min(models, key=lambda kk: abs(int(kk) - k))
    d = models[key]
    params = torch.tensor(d["params"], dtype=torch.float32, device=device)
    norm = torch.tensor(d["mean"] + d["std"], dtype=torch.float32, device=device)
    if params.numel() != kc.MLP_NPARAMS or norm.numel() != 8:
        raise ValueError(f"{path}: wrong parameter count")
    return params, norm


def init_params(seed: int = 0) -> np.ndarray:
    """He initialisation: weights ~ N(0, 2/fan_in), biases 0 (layout of
    include/kclique.h)."""
    r = np.random.default_rng(seed)
    H, NI = kc.MLP_HIDDEN, kc.MLP_IN
    parts = [r.normal(0, math.sqrt(2.0 / NI), H * NI), np.zeros(H), r.normal(0, math.sqrt(2.0 / H), H * H),
             np.zeros(H), r.normal(0, math.sqrt(1.0 / H), H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def collect(row_ptr, col_idx, k: int, device):
    """Runs BitCol with per-root logging; returns (features[R, 4], work[R],
    count) for the roots (d+ >= k-1)."""
    import torch
    rp = torch.as_tensor(row_ptr).to(device)
    ci = torch.as_tensor(col_idx).to(device)
    c, st = kc.count(rp, ci, k, "color", root_logs=True)
    lg = st["root_logs"]
    f = lg["features"].cpu().numpy()
    wk = lg["work"].cpu().numpy().astype(np.float64)
    roots = f[:, 0] >= k - 1
    return f[roots].astype(np.float64), wk[roots], c


def features_to_x(f: np.ndarray, mean, std) -> np.ndarray:
    return ((np.log1p(f) - mean) / std).astype(np.float32)


def train(X: np.ndarray, y: np.ndarray, device, steps: int = 4000, batch: int = 4096, lr: float = 2e-3,
          seed: int = 0, log_every: int = 500):
    """Adam on minibatches drawn with a fixed seed; returns params (tensor)
    and the loss history."""
    import torch
    r = np.random.default_rng(seed)
    P = torch.tensor(init_params(seed), device=device)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    Xd = torch.tensor(X, device=device)
    yd = torch.tensor(y.astype(np.float32), device=device)
    hist = []
    n = X.shape[0]
    for t in range(1, steps + 1):
        idx = torch.tensor(r.integers(0, n, min(batch, n)), device=device)
        # cosine decay of the step size
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * (t - 1) / steps))
        loss, _ = kc.mlp_train_step(P, Xd[idx].contiguous(), yd[idx].contiguous(), m, v, t=t, lr=lr_t)
        if t % log_every == 0 or t == 1:
            hist.append((t, float(loss.item())))
            print(f"  step {t}: minibatch mse {hist[-1][1]:.4f}", flush=True)
    return P, hist


def spearman(a: np.ndarray, b: np.ndarray) -> float:
    """Spearman rank correlation (average ranks for ties)."""
    from scipy.stats import rankdata
    ra = rankdata(a).astype(np.float64)
    rb = rankdata(b).astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / math.sqrt((ra * ra).sum() * (rb * rb).sum()))


def train_for_k(k: int, dev, seed: int = 0) -> dict:
    import torch

    import graphgen
    feats, targets, meta = [], [], []
    for cfg, scale in TRAIN_SETS[k]:
        w = graphgen.workload(cfg, scale=scale)
        t0 = time.time()
        f, wk, c = collect(*w.graphs[0], k, dev)
        torch.cuda.synchronize()
        print(f"{w.name} k={k}: {len(wk)} roots, {c} cliques, logged in {time.time() - t0:.1f}s", flush=True)
        feats.append(f)
        targets.append(np.log1p(wk))
        meta.append(dict(workload=w.name, k=k, roots=int(len(wk)), count=int(c)))
    F = np.concatenate(feats)
    Y = np.concatenate(targets)
    # cap the set size: every root in the heaviest tenth plus a sample of the rest
    r = np.random.default_rng(seed + 1)
    q = np.quantile(Y, 0.9)
    heavy = np.nonzero(Y > q)[0]
    light = np.nonzero(Y <= q)[0]
    light = r.choice(light, size=min(len(light), 400_000), replace=False)
    sel = np.concatenate([heavy, light])
    F, Y = F[sel], Y[sel]
    lf = np.log1p(F)
    mean = lf.mean(axis=0)
    std = lf.std(axis=0) + 1e-6
    X = features_to_x(F, mean, std)
    perm = r.permutation(len(Y))
    n_val = len(Y) // 10
    val, tr = perm[:n_val], perm[n_val:]
    print(f"k={k}: training on {len(tr)} roots, validating on {len(val)}", flush=True)
    P, hist = train(X[tr], Y[tr], dev, seed=seed)
    pred = kc.mlp_forward(P, torch.tensor(X[val], device=dev)).cpu().numpy()
    mse = float(np.mean((pred - Y[val]) ** 2))
    rho = spearman(pred, Y[val])
    print(f"k={k} validation: mse {mse:.4f} (target variance {np.var(Y[val]):.4f}), spearman {rho:.4f}", flush=True)
    return dict(k=k, params=[float(x) for x in P.cpu().numpy()], mean=[float(x) for x in mean],
                std=[float(x) for x in std], train_sets=meta, loss_history=hist,
                validation=dict(mse=mse, target_var=float(np.var(Y[val])), spearman=rho, rows=int(n_val)),
                features=["log1p d+", "log1p core", "log1p colors", "log1p |E_u|"], target="log1p words")


def main(argv=None):
    import torch
    dev = torch.device("cuda:0")
    out = argv[0] if argv else MODEL_PATH
    models = {str(k): train_for_k(k, dev) for k in sorted(TRAIN_SETS)}
    with open(out, "w") as f:
        json.dump(dict(models=models), f)
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
