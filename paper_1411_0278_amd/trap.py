"""Checkpointed trap runs over the C ABI (driver only; the arithmetic is in libmbstokes).

A run advances the spheres with mbs_step in segments of `checkpoint_every` steps and after each
segment writes a checkpoint: step count, positions, orientations, the integrator's history
(previous step's V, Omega x p and Sigma) and the run parameters, as a NumPy .npz file. `resume`
continues from a checkpoint; because the kernels are deterministic and the history is carried
over, a run of N steps and a run of N1 steps + resume + N2 steps give identical results.
"""
from __future__ import annotations

import numpy as np

CHECKPOINT_KEYS = ("step", "R", "p", "hist", "k_trap", "slip_coef", "dt", "order")


def save_checkpoint(path, step, R, p, hist, k_trap, slip_coef, dt, order):
    np.savez(path, step=np.int64(step), R=np.asarray(R, dtype=np.float64), p=np.asarray(p, dtype=np.float64),
             hist=np.asarray(hist, dtype=np.float64), k_trap=np.float64(k_trap),
             slip_coef=np.asarray(slip_coef, dtype=np.float64), dt=np.float64(dt), order=np.int64(order))


def load_checkpoint(path):
    with np.load(path) as z:   # plain arrays only (no pickled objects)
        return {k: z[k].copy() for k in CHECKPOINT_KEYS}


def run(ctx, R, p, k_trap, slip_coef, dt, nsteps, order=2, checkpoint_every=0, path=None, start=None):
    """Advance R, p (float64 CUDA tensors, updated in place) by nsteps. start: a checkpoint dict to
    continue from (its history is used). Returns (per-step stats, history tensor, steps done)."""
    import torch
    n = R.shape[0]
    hist = torch.zeros(11 * n, dtype=torch.float64, device=R.device)
    valid = False
    step0 = 0
    if start is not None:
        hist.copy_(torch.as_tensor(start["hist"], device=R.device))
        valid = True
        step0 = int(start["step"])
    stats = []
    seg = checkpoint_every if checkpoint_every > 0 else nsteps
    done = 0
    while done < nsteps:
        todo = min(seg, nsteps - done)
        st, _ = ctx.mbs_step(R, p, k_trap, slip_coef, dt, todo, order=order, allow_noconv=True,
                             hist=hist, hist_valid=valid)
        stats += st
        valid = True
        done += todo
        if path and checkpoint_every > 0:
            save_checkpoint(path, step0 + done, R.cpu().numpy(), p.cpu().numpy(), hist.cpu().numpy(),
                            k_trap, slip_coef, dt, order)
    return stats, hist, step0 + done


def resume(ctx, path, nsteps, device="cuda:0"):
    """Continue the run stored at `path` by nsteps; returns (R, p, stats, hist, step)."""
    import torch
    ck = load_checkpoint(path)
    R = torch.as_tensor(ck["R"]).to(device)
    p = torch.as_tensor(ck["p"]).to(device)
    stats, hist, step = run(ctx, R, p, float(ck["k_trap"]), tuple(ck["slip_coef"]), float(ck["dt"]), nsteps,
                            int(ck["order"]), start=ck)
    return R, p, stats, hist, step
