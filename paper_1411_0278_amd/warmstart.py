"""Training pipeline of the learned warm start (driver over the C ABI; all arithmetic in libmbstokes).

1. Data: solve trap workloads of 10^4 spheres at the benchmark density (cube side 199.6, seeds
   0..K-1) to a binary64 residual of 1e-10; every sphere is one sample: its neighbourhood features
   (80 geometric values, or 160 with the neighbours' one-body stresslets gamma b_j) and the target
   Sigma - gamma b (the many-body part of its flow stresslet beyond the one-body guess).
2. Training: Adam on the GPU (bfloat16 operands, float32 accumulation), mean squared error.
3. Use: MBS_GUESS_LEARNED starts GMRES from gamma b + net(features).

    python -m paper_1411_0278_amd.warmstart --configs 200 --epochs 10 --out weights.bin
"""
from __future__ import annotations

import argparse
import sys
import time

N_TRAIN = 10_000
SIDE_TRAIN = 430.0 * (N_TRAIN / 100_000) ** (1.0 / 3.0)   # same number density as N = 1e5 in side 430


def training_set(ctx, seeds, n=N_TRAIN, side=SIDE_TRAIN, tol=1e-10, log=None, feature_sets=(0,)):
    """Features {set: [M, in]} and targets [M, 5] (float32 device tensors) from converged solves.
    Feature set 0 is the neighbourhood geometry (80 values); set 1 adds each neighbour's one-body
    stresslet gamma b_j (160 values), b the right-hand side the library forms for the same spheres."""
    import torch

    from . import inputs, mbstokes
    feats = {fs: [] for fs in feature_sets}
    targets = []
    t0 = time.perf_counter()
    prm = dict(precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_DIAG, tol=tol)
    old = {k: getattr(ctx.params, k) for k in prm}
    ctx.set_params(**prm)
    if mbstokes.MBS_FEATURES_GEOMETRY_RHS in feature_sets:
        ctx.mbs_warmstart_features(mbstokes.MBS_FEATURES_GEOMETRY_RHS)  # (no network yet)
    try:
        for k, seed in enumerate(seeds):
            w = inputs.trap_workload(n, side, int(seed))
            d = mbstokes.to_device(w, "cuda:0")
            Sigma = torch.empty((n, 5), dtype=torch.float64, device="cuda:0")
            ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None, Sigma=Sigma)
            targets.append(ctx.mbs_warmstart_target(d["R"], Sigma, d["v2s"], None, d["Fe"], None))
            for fs in feature_sets:
                if fs == mbstokes.MBS_FEATURES_GEOMETRY:
                    feats[fs].append(ctx.mbs_features(d["R"], d["p"]))
                else:
                    b = ctx.mbs_rhs(d["R"], d["v2s"], None, d["Fe"], None)
                    feats[fs].append(ctx.mbs_features_ex(d["R"], d["p"], b))
            if log and (k + 1) % 25 == 0:
                log(f"warmstart: {k + 1} training solves done ({time.perf_counter() - t0:.1f} s)")
    finally:
        ctx.set_params(**old)
    return {fs: torch.cat(v) for fs, v in feats.items()}, torch.cat(targets)


def surrogate_error(ctx, d, Sigma_star, guess):
    """||Sigma^0 - Sigma*|| / ||Sigma*|| of an initial guess (reporting only)."""
    s0 = ctx.mbs_initial_guess(d["R"], guess, d["p"], d["v2s"], None, d["Fe"], None)
    return float((s0 - Sigma_star).norm() / Sigma_star.norm())


def train_pipeline(ctx, n_configs=200, n_val=10, epochs=10, batch=4096, lr=1e-3, seed=0, log=None,
                   feature_sets=(0,), weights=None, n=N_TRAIN, side=SIDE_TRAIN):
    """Generate data (last n_val configurations held out) and train one network per feature set;
    `weights` maps a feature set to a file the trained parameters are saved to. The context keeps the
    last network trained. Returns {feature set: report}."""
    import torch
    seeds = list(range(n_configs))
    t0 = time.perf_counter()
    X, T = training_set(ctx, seeds, n=n, side=side, log=log, feature_sets=feature_sets)
    t_data = time.perf_counter() - t0
    n_tr = (n_configs - n_val) * n
    Ttr, Tva = T[:n_tr].contiguous(), T[n_tr:].contiguous()
    out = {}
    for fs in feature_sets:
        Xtr, Xva = X[fs][:n_tr].contiguous(), X[fs][n_tr:].contiguous()
        ctx.mbs_warmstart_features(fs)
        ctx.mbs_warmstart_init(seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hist = ctx.mbs_warmstart_train(Xtr, Ttr, epochs=epochs, batch=batch, lr=lr, seed=seed)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        val = {}
        if Xva.shape[0]:
            pred = ctx.mbs_warmstart_forward(Xva)
            val = {"val_mse": float(((pred - Tva) ** 2).mean()),
                   "val_target_ms": float((Tva ** 2).mean())}
        if weights and fs in weights:
            ctx.mbs_warmstart_save(weights[fs])
        out[fs] = {"feature_set": fs, "inputs": int(Xtr.shape[1]), "samples": int(n_tr),
                   "val_samples": int(Xva.shape[0]), "epochs": epochs, "batch": batch, "lr": lr,
                   "loss_history": hist, "data_seconds": t_data, "train_seconds": t_train, **val}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--configs", type=int, default=200)
    ap.add_argument("--val", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--features", type=int, default=0, choices=(0, 1),
                    help="0: neighbourhood geometry (80 inputs); 1: geometry and the neighbours' gamma b (160)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    from . import mbstokes
    ctx = mbstokes.Context(0)
    rep = train_pipeline(ctx, a.configs, a.val, a.epochs, a.batch, a.lr, a.seed,
                         log=lambda s: print(s, file=sys.stderr, flush=True), feature_sets=(a.features,),
                         weights={a.features: a.out})
    print(rep)


if __name__ == "__main__":
    main()
