"""Warm-start pipeline on top of the C ABI: training pairs from plain
refinement, network training, and the time-to-PSNR comparison of warm-started
versus plain refinement at equal final PSNR.

Every numerical step is a library call (allocation, features, refinement,
targets, training, warm start); this module only sequences them.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import (MLP, Context, Grid, Params, _check, _lib, _vp, allocate, features, loss_grad,
               mlp_train, refine, targets, warmstart)


def clone(ctx: Context, p: Params) -> Params:
    """A new parameter set holding a device copy of p's parameters."""
    q = Params(ctx, p.n)
    _check(_lib.gve_params_copy_from_device(ctx.handle, q.handle, _vp(p.device_ptr())), ctx.handle)
    return q


def training_pairs(ctx: Context, field, grid: Grid, budget: int, seed: int, iters: int):
    """(features [n,16], targets [n,11]) of one encoding: allocation -> `iters`
    plain refinement iterations."""
    P, info = allocate(ctx, field, grid, budget, seed)
    X = features(ctx, P, field, grid, info["n_detail"], info["g99"])
    A = clone(ctx, P)
    refine(ctx, P, field, grid, iters, want_losses=False)
    T = targets(ctx, A, P)
    A.close()
    P.close()
    return X, T


def psnr(loss, n_voxels):
    return 10.0 * math.log10(n_voxels / loss) if loss > 0 else float("inf")


def plain_run(ctx: Context, field, grid: Grid, budget: int, seed: int, iters: int):
    """Plain refinement: returns dict with wall seconds, loss history and final PSNR."""
    import torch

    M = grid.nx * grid.ny * grid.nz
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, info = allocate(ctx, field, grid, budget, seed)
    t_alloc = time.perf_counter() - t0
    losses = refine(ctx, P, field, grid, iters)
    final = loss_grad(ctx, P, field, grid)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.close()
    return {"seconds": wall, "alloc_seconds": t_alloc, "iterations": iters,
            "psnr_start": psnr(losses[0], M), "psnr_final": psnr(final, M), "loss_final": final,
            "info": info}


def next_call_size(losses, target_loss: float, rate, most: int):
    """Iterations for the next refinement call, and the updated rate.

    `losses` are the previous call's losses (before each of its updates) and
    `rate` the last known decrease of log(loss) per iteration.  The remaining
    iterations are predicted from the most recent rate (the loss's decrease
    slows as refinement converges, so the prediction falls short rather than
    overshoots) and rounded down; at least one."""
    if len(losses) >= 2 and losses[0] > losses[-1] > 0:
        rate = (math.log(losses[0]) - math.log(losses[-1])) / (len(losses) - 1)
    if not rate or not 0 < losses[-1] < math.inf or not target_loss > 0:
        return most, rate
    # updates still needed from the state of losses[-1]; the call's last
    # update is already done, and a call of n records the state after n - 1
    left = (math.log(losses[-1]) - math.log(target_loss)) / rate
    return int(max(1, min(most, math.floor(left)))), rate


def warm_run(ctx: Context, mlp: MLP, field, grid: Grid, budget: int, seed: int, target_loss: float,
             max_iters: int, chunk: int = 0, first: int = 64):
    """Warm-started refinement until the loss reaches target_loss (or max_iters).

    Refines in calls that each return the loss before each of their updates,
    so the first loss at or below the target gives the iteration count; the
    rest of that call's iterations are extra work that the wall time
    includes.  chunk > 0: calls of `chunk` iterations.  chunk = 0: the first
    call runs `first` iterations and each later one as many as the loss's
    recent rate of decrease predicts are still needed (`next_call_size`), so
    that few calls are made and the last one ends near the target."""
    import torch

    M = grid.nx * grid.ny * grid.nz
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, info = allocate(ctx, field, grid, budget, seed)
    applied, L = warmstart(ctx, mlp, P, field, grid, info["n_detail"], info["g99"])
    t_warm = time.perf_counter() - t0
    it = 0
    cur = L[applied] if applied else L[0]
    start_loss = cur
    if cur > target_loss:
        size, rate = (chunk if chunk > 0 else first), None
        while it < max_iters:
            step = min(size, max_iters - it)
            losses = refine(ctx, P, field, grid, step)
            # losses[j] is the loss before update j: stop at the first that meets the target
            hit = np.nonzero(losses <= target_loss)[0]
            if hit.size:
                it += int(hit[0])
                cur = float(losses[hit[0]])
                break
            it += step
            if chunk <= 0:
                size, rate = next_call_size(losses, target_loss, rate, first)
        else:
            cur = loss_grad(ctx, P, field, grid)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.close()
    return {"seconds": wall, "warm_seconds": t_warm, "iterations": it, "applied": applied,
            "alloc_losses": [x if np.isfinite(x) else None for x in L.tolist()],
            "psnr_start": psnr(start_loss, M),
            "psnr_final": psnr(cur, M), "reached": cur <= target_loss}


def train_network(ctx: Context, pairs, epochs=20, batch=4096, lr=1e-3, seed=0):
    """Concatenate (X, T) pairs and train a fresh network; returns (mlp, epoch losses)."""
    import torch

    X = torch.cat([p[0] for p in pairs])
    T = torch.cat([p[1] for p in pairs])
    mlp = MLP(ctx, seed=seed)
    hist = mlp_train(ctx, mlp, X.contiguous(), T.contiguous(), epochs, batch, lr, seed)
    return mlp, hist, int(X.shape[0])
