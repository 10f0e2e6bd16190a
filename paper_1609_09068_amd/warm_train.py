"""Training the starting-guess network on ranks the method itself produces.

For each training graph (the web-like recipe at 100k vertices / 1M edges,
seeds 4001...): partition, plan, solve componentwise in FP64 to a 1e-12
certificate, then take every SCC vertex's features (pr_warm_features) and
its target log(R_v / s_C).  The network is trained on the GPU by the
library's own kernels (pr_mlp_train_step: BF16 matrix-core forward and
backward, Adam), on random batches drawn on the device.

    python -m paper_1609_09068_amd.warm_train --graphs 200 --steps 20000 \\
        --out paper_1609_09068_amd/data/warm_web.prmlp
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEFAULT_NET = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "warm_web.prmlp")


def log(*a):
    print("[warm_train]", *a, file=sys.stderr, flush=True)


def graph_samples(pr, torch, g, c=0.85, eps=1e-12):
    """(features [k, 4], targets [k]) of the SCC vertices of graph g, on the device."""
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col)
    W = torch.ones(g.n, dtype=torch.float64, device="cuda")
    R = torch.empty_like(W)
    pr.pr_solve(lv, c, W, R, eps=eps, precision=pr.PR_PREC_FP64)
    F, S, M = pr.warm_features(lv, c, W)
    m = M.bool()
    t = torch.log(R[m] / S[m].double()).float()
    return F[m].contiguous(), t.contiguous()


def collect(pr, torch, seeds, c=0.85):
    sys.path.insert(0, ROOT)
    from graphgen import config_graph

    Xs, ts = [], []
    t0 = time.perf_counter()
    for i, sd in enumerate(seeds):
        g = config_graph("c4_train_100k", seed=sd)
        X, t = graph_samples(pr, torch, g, c)
        Xs.append(X)
        ts.append(t)
        if (i + 1) % 10 == 0 or i + 1 == len(seeds):
            log(f"graphs {i + 1}/{len(seeds)}: {sum(len(x) for x in ts)} rows, {time.perf_counter() - t0:.1f} s")
    return torch.cat(Xs), torch.cat(ts)


def train(pr, torch, X, t, steps=20000, batch=8192, lr=3e-3, lr_end=3e-4, seed=0, net=None, log_every=2000):
    """Adam on random batches; the learning rate decays geometrically from lr to lr_end."""
    net = net or pr.Mlp.create(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = X.shape[0]
    hist = []
    for s in range(steps):
        rate = lr * (lr_end / lr) ** (s / max(steps - 1, 1))
        sel = torch.randint(0, n, (batch,), device="cuda", generator=gen)
        loss = net.train_step(X[sel].contiguous(), t[sel].contiguous(), rate)
        if s % log_every == 0 or s + 1 == steps:
            hist.append((s, loss))
            log(f"step {s}: batch mse {loss:.5f} (lr {rate:.2e})")
    return net, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=200)
    ap.add_argument("--first-seed", type=int, default=4001)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--c", type=float, default=0.85)
    ap.add_argument("--out", default=DEFAULT_NET)
    args = ap.parse_args()

    import torch

    sys.path.insert(0, ROOT)
    import paper_1609_09068_amd as pr

    X, t = collect(pr, torch, range(args.first_seed, args.first_seed + args.graphs), args.c)
    log(f"training rows {X.shape[0]}, target mean {t.mean().item():.4f} std {t.std().item():.4f}")
    net, hist = train(pr, torch, X, t, args.steps, args.batch, args.lr)
    _, full = net.grad(X[: min(len(X), 2_000_000)].contiguous(), t[: min(len(t), 2_000_000)].contiguous())
    base = float(((t - t.mean()) ** 2).mean())
    log(f"mse on the first 2M rows {full:.5f} (variance of the target {base:.5f})")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    log(f"saved {args.out}")


if __name__ == "__main__":
    main()
