"""The learned warm start against plain refinement (what the network gains).

Pairs (allocation -> 300 plain iterations) from six seeded 128^3 fronts fields
train the network on the device; on two unseen seeds the warm-started
refinement must reach the plain schedule's final PSNR in fewer iterations,
and the warm start must never make the allocation worse (its fallback).
"""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_reaches_plain_psnr_in_fewer_iterations():
    import torch

    import paper_2608_14112_amd as g
    import paper_2608_14112_amd.warm as W
    from synth import fields as S

    n, iters = 128, 300
    budget = n ** 3 // 512
    grid = g.Grid(n, n, n)
    ctx = g.Context(k=3.0, lr=8e-3, ell_min=math.log(0.25), ell_max=math.log(n / 16))
    pairs = []
    for s in range(6):
        f = S.fronts_field(n, 100 + s, device="cuda")
        pairs.append(W.training_pairs(ctx, f, grid, budget, 100 + s, iters))
    mlp, hist, _ = W.train_network(ctx, pairs, epochs=30, batch=2048, lr=1e-3, seed=1)
    assert hist[-1] < hist[0]
    gains = []
    for es in (999, 998):
        f = S.fronts_field(n, es, device="cuda")
        plain = W.plain_run(ctx, f, grid, budget, es, iters)
        warm = W.warm_run(ctx, mlp, f, grid, budget, es, plain["loss_final"], iters)
        print(f"seed {es}: plain {iters} it -> {plain['psnr_final']:.2f} dB; warm "
              f"{warm['iterations']} it (start {warm['psnr_start']:.2f} dB vs "
              f"{plain['psnr_start']:.2f}), applied {warm['applied']}", flush=True)
        assert warm["psnr_start"] >= plain["psnr_start"] - 1e-9   # never worse
        assert warm["reached"]
        gains.append(1 - warm["iterations"] / iters)
    assert min(gains) > 0.0, gains
