"""Training driver of the learned body-mobility network (argument marshalling and
batching only; labels, features, forward, backward and Adam run in libarb).

Data: independent bacterium poses above the wall (``workloads.bacterium_poses``),
labelled by the exact block build of Sec. 3.1 (``arb_body_mobility``).
"""
from __future__ import annotations

import numpy as np

from . import arb
from . import workloads as W


def make_dataset(n_bact: int, seed: int = 5, chunk: int = 8192, device: int = 0):
    """Features (2 n_bact x 7) and labels (2 n_bact x 21), float32 host arrays."""
    Xs, Ts = [], []
    done = 0
    k = 0
    while done < n_bact:
        m = min(chunk, n_bact - done)
        wl = W.bacterium_poses(m, seed=seed + 1000 * k)
        ctx = arb.context_for(wl, precision=arb.ARB_FP64, device=device)
        try:
            _, T = arb.arb_body_mobility(ctx)
            X = arb.arb_mlp_features(ctx)
        finally:
            arb.arb_destroy(ctx)
        Xs.append(X)
        Ts.append(T)
        done += m
        k += 1
    return np.vstack(Xs), np.vstack(Ts)


def scaling(X, T):
    """Standardisation constants from a training set: (mu_x, sd_x, mu_y, sd_y)."""
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    return (X.mean(0).astype(np.float32), np.maximum(X.std(0), 1e-3).astype(np.float32),
            T.mean(0).astype(np.float32), np.maximum(T.std(0), 1e-6).astype(np.float32))


def load_model(ctx, params, scale):
    arb.arb_mlp_set_scaling(ctx, *scale)
    arb.arb_mlp_set_params(ctx, params)


def train(ctx, X, T, epochs: int = 30, batch: int = 4096, lr: float = 2e-3, seed: int = 7,
          lr_final: float = 1e-3, log=None):
    """Adam on the GPU over shuffled batches, learning rate on a cosine from lr
    down to lr * lr_final; returns the per-epoch loss of the last batch
    (computed before its step, on standardised outputs)."""
    import math

    import torch

    dev = torch.device("cuda", 0)
    Xd = torch.tensor(np.asarray(X, np.float32), device=dev)
    Td = torch.tensor(np.asarray(T, np.float32), device=dev)
    n = Xd.shape[0]
    rng = np.random.default_rng(seed)
    stream = torch.cuda.Stream()
    hist = []
    lr0 = lr
    for ep in range(epochs):
        lr = lr0 * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + math.cos(math.pi * ep / epochs)))
        perm = torch.tensor(rng.permutation(n), device=dev)
        with torch.cuda.stream(stream):
            for s0 in range(0, n - batch + 1, batch):
                idx = perm[s0:s0 + batch]
                xb = Xd.index_select(0, idx).contiguous()
                tb = Td.index_select(0, idx).contiguous()
                last = s0 + 2 * batch > n
                loss = arb.arb_mlp_train_step_dev(ctx, batch, xb, tb, lr, want_loss=last,
                                                  stream=stream.cuda_stream)
        torch.cuda.synchronize()
        hist.append(loss)
        if log:
            log(f"epoch {ep}: loss {loss:.3e} lr {lr:.2e}")
    return hist
