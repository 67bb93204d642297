"""The neural surrogate of Sec. 4.3, retrained on this library's exact sPAM states and
compared with them.

The paper replaces the numerical solution of Eq. 1 by a 2-32-2 perceptron (ReLU, He
initialisation) from (strain, unit length) to the sPAM parameters (m, phi), trained on
40,000 solved states with an 80/10/10 split, and reports a mean squared error of 0.003
on normalized outputs.  Here the states come from ``vine_spam_solve`` (Eq. 1 solved
exactly on the GPU, one wave per state); the network is trained on the host (plain
mini-batch Adam in numpy: a fit done once, like the force-law tables) and evaluated on
the GPU by ``vine_mlp_forward``.

Readings: the samples are uniform in unit length over [20, 80] mm and in strain over
[0, slack strain) of that length (the paper draws m uniformly; uniform strain covers the
network's input domain evenly); inputs are scaled as (eps / 0.5, (l0 - 0.02) / 0.06) and
outputs as (m / 0.5, phi / (pi / 2)); the weights of the epoch with the lowest validation
error are kept.

Run ``python -m paper_2509_15180_amd.surrogate`` for one training and measurement as a
JSON line.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np

L0_LO, L0_HI = 0.02, 0.08


def scale_in(eps, l0):
    return np.stack([np.asarray(eps) / 0.5, (np.asarray(l0) - L0_LO) / (L0_HI - L0_LO)], -1)


def unscale_out(y):
    return y[..., 0] * 0.5, y[..., 1] * (math.pi / 2)


def samples(n: int, seed: int = 0, params=None):
    """n exact states: (eps, l0, m, phi, G) columns, drawn as the module describes."""
    from . import vinesim as V
    rng = np.random.default_rng(seed)
    l0 = rng.uniform(L0_LO, L0_HI, n)
    slack = V.spam_solve(np.full(n, 10.0), l0, params)[:, 3]
    eps = rng.uniform(0.0, 1.0, n) * slack
    st = V.spam_solve(eps, l0, params)
    return np.column_stack([eps, l0, st[:, 0], st[:, 1], st[:, 2]])


def pack(W1, b1, W2, b2) -> np.ndarray:
    """The layout of vine_mlp_forward: W1 [32][2], b1 [32], W2 [2][32], b2 [2]."""
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2])


def unpack(w):
    return w[:64].reshape(32, 2), w[64:96], w[96:160].reshape(2, 32), w[160:162]


def forward(w, X):
    W1, b1, W2, b2 = unpack(w)
    return np.maximum(X @ W1.T + b1, 0.0) @ W2.T + b2


def train(X, Y, Xv, Yv, epochs: int = 300, batch: int = 256, lr: float = 2e-3, seed: int = 0):
    """Mini-batch Adam on the mean squared error; the weights of the best validation
    epoch and the per-epoch validation errors."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, math.sqrt(2.0 / 2), (32, 2))
    W2 = rng.normal(0.0, math.sqrt(2.0 / 32), (2, 32))
    params = [W1, np.zeros(32), W2, np.zeros(2)]
    m1 = [np.zeros_like(p) for p in params]
    m2 = [np.zeros_like(p) for p in params]
    step, best, best_w, hist = 0, np.inf, pack(*params), []
    for ep in range(epochs):
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))
        order = rng.permutation(len(X))
        for s in range(0, len(X), batch):
            idx = order[s:s + batch]
            x, y = X[idx], Y[idx]
            W1, b1, W2, b2 = params
            z = x @ W1.T + b1
            h = np.maximum(z, 0.0)
            out = h @ W2.T + b2
            g = 2.0 * (out - y) / (len(x) * 2)
            gW2, gb2 = g.T @ h, g.sum(0)
            gh = (g @ W2) * (z > 0.0)
            gW1, gb1 = gh.T @ x, gh.sum(0)
            step += 1
            for p, gp, a, b in zip(params, (gW1, gb1, gW2, gb2), m1, m2):
                a *= 0.9
                a += 0.1 * gp
                b *= 0.999
                b += 0.001 * gp * gp
                p -= rate * (a / (1 - 0.9 ** step)) / (np.sqrt(b / (1 - 0.999 ** step)) + 1e-8)
        v = float(np.mean((forward(pack(*params), Xv) - Yv) ** 2))
        hist.append(v)
        if v < best:
            best, best_w = v, pack(*params)
    return best_w, hist


def spam_G(m, phi, R_c: float = 0.005):
    """G = F_t / P_act of Eq. 1d."""
    return math.pi * R_c ** 2 * (1.0 - 2.0 * m) / (2.0 * m * np.cos(phi) ** 2)


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=40000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--bench", type=int, default=1 << 20, help="states for the throughput test")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    import torch

    from . import vinesim as V
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    D = samples(args.samples, args.seed)
    t_data = time.perf_counter() - t0
    rng = np.random.default_rng(args.seed + 1)
    perm = rng.permutation(len(D))
    n_tr, n_va = int(0.8 * len(D)), int(0.1 * len(D))
    tr, va, te = perm[:n_tr], perm[n_tr:n_tr + n_va], perm[n_tr + n_va:]
    X = scale_in(D[:, 0], D[:, 1])
    Y = np.column_stack([D[:, 2] / 0.5, D[:, 3] / (math.pi / 2)])
    t1 = time.perf_counter()
    w, hist = train(X[tr], Y[tr], X[va], Y[va], epochs=args.epochs, seed=args.seed)
    t_train = time.perf_counter() - t1
    y_gpu = V.mlp_forward(w, X[te])
    mse = float(np.mean((y_gpu - Y[te]) ** 2))
    m, phi = unscale_out(y_gpu)
    G0 = V.spam_solve(np.zeros(len(te)), D[te, 1])[:, 2]
    dG = np.abs(spam_G(m, phi) - D[te, 4]) / G0
    # throughput: the exact states against the surrogate, same inputs
    rb = np.random.default_rng(args.seed + 2)
    l0b = rb.uniform(L0_LO, L0_HI, args.bench)
    eb = rb.uniform(0.0, 0.15, args.bench)
    V.spam_solve(eb[:64], l0b[:64])
    a = time.perf_counter()
    V.spam_solve(eb, l0b)
    t_exact = time.perf_counter() - a
    Xb = scale_in(eb, l0b)
    V.mlp_forward(w, Xb[:64])
    a = time.perf_counter()
    V.mlp_forward(w, Xb)
    t_net = time.perf_counter() - a
    rec = {"study": "sPAM surrogate (2-32-2 ReLU) against exact Eq. 1 states",
           "samples": args.samples, "split": "80/10/10", "epochs": args.epochs,
           "test_mse_normalized": mse, "best_val_mse": float(min(hist)),
           "force_error_over_G0": {"median": float(np.median(dG)),
                                   "p99": float(np.quantile(dG, 0.99)), "max": float(dG.max())},
           "s_data_gpu": t_data, "s_train_host": t_train,
           "bench_states": args.bench, "exact_states_per_s": args.bench / t_exact,
           "surrogate_states_per_s": args.bench / t_net}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
