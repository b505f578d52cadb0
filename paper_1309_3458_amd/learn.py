"""Training of the hit-count predictor on counts the exact matcher produces.

Labels are y = log1p(count_j), where count_j is the exact number of
subscriptions update j meets (ddm_count, i.e. the plain count traversal /
BITS).  Features come from ddm_features; the network is trained with the
library's own GPU kernels (ddm_predictor_train).  The sizing margin delta is
the 99th percentile of the held-out residuals y - yhat, so that about 1% of
held-out updates overflow their slots.

Training draws are uniform placements like the paper's workloads
(Sec. V: N extents, overlap degree alpha) extended to d in {1, 2, 3}, with
seeds >= 100 so that they never coincide with an evaluation draw.

    python -m paper_1309_3458_amd.learn --out predictor.ddmp
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np

from . import workloads as W


def draw_specs(n_inst: int, seed: int = 100, n_lo: float = 1e3, n_hi: float = 1e6,
               a_lo: float = 0.01, a_hi: float = 100.0, dims=(1, 2, 3)):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_inst):
        N = 2 * int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) / 2))
        d = int(dims[int(rng.integers(0, len(dims)))])
        alpha = float(math.exp(rng.uniform(math.log(a_lo), math.log(a_hi))))
        specs.append(W.BatchSpec(N=max(N, 2), d=d, alpha=alpha, seed=(seed, i)))
    return specs


def dataset(specs, per_instance: int = 20000, seed: int = 7):
    """(X [S,18], Y [S]) as host arrays: GPU features and log1p(exact counts)."""
    import torch

    from . import build, count, features

    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for spec in specs:
        inst = W.instance_from_spec(spec)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        take = np.sort(rng.choice(inst.m, size=min(per_instance, inst.m), replace=False))
        u_lo, u_hi = dev(inst.u_lo[:, take]), dev(inst.u_hi[:, take])
        t = build(dev(inst.s_lo), dev(inst.s_hi))
        cnt, _ = count(t, u_lo, u_hi)
        xs.append(features(t, u_lo, u_hi).cpu().numpy())
        ys.append(np.log1p(cnt.cpu().numpy().astype(np.float64)).astype(np.float32))
        t.free()
    return np.concatenate(xs), np.concatenate(ys)


def train_predictor(n_inst: int = 48, per_instance: int = 20000, epochs: int = 30,
                    batch: int = 4096, lr: float = 2e-3, seed: int = 100, quantile: float = 0.99,
                    verbose: bool = False):
    """Train on fresh uniform draws; returns (predictor, report dict)."""
    import torch

    from . import Predictor

    t0 = time.time()
    specs = draw_specs(n_inst, seed=seed)
    X, Y = dataset(specs, per_instance)
    S = X.shape[0]
    order = np.random.default_rng(seed).permutation(S)
    X, Y = X[order], Y[order]
    n_val = max(1, S // 10)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Xtr, Ytr = dev(X[n_val:]), dev(Y[n_val:])
    Xva, Yva = dev(X[:n_val]), dev(Y[:n_val])
    t_data = time.time() - t0
    p = Predictor(seed)
    t1 = time.time()
    l1 = p.train(Xtr, Ytr, batch=batch, epochs=epochs, lr=lr)
    l2 = p.train(Xtr, Ytr, batch=batch, epochs=max(1, epochs // 3), lr=lr / 5)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    yhat = p.forward(Xva).cpu().numpy().astype(np.float64)
    yv = Yva.cpu().numpy().astype(np.float64)
    res = yv - yhat
    delta = float(np.quantile(res, quantile))
    p.set_params(None, delta)
    rep = {
        "samples": int(S), "train_samples": int(S - n_val), "val_samples": int(n_val),
        "epochs": int(epochs + max(1, epochs // 3)), "loss_first": float(l1[0]),
        "loss_last": float(l2[-1]), "val_mae_log1p": float(np.mean(np.abs(res))),
        "delta": delta, "val_under_rate": float(np.mean(res > delta)),
        "data_s": round(t_data, 2), "train_s": round(t_train, 2),
    }
    if verbose:
        print(rep, flush=True)
    return p, rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="predictor.ddmp")
    ap.add_argument("--instances", type=int, default=48)
    ap.add_argument("--epochs", type=int, default=30)
    args = ap.parse_args()
    p, rep = train_predictor(args.instances, epochs=args.epochs, verbose=True)
    p.save(args.out)


if __name__ == "__main__":
    main()
