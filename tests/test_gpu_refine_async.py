"""Refinement with asynchronous binning.

Inside gve_refine only the first iteration waits for the device to size the
pair buffers; later iterations bin into buffers of that capacity with every
count kept on the device.  With deterministic gradient sums the pair lists,
and therefore the whole trajectory, are identical to those of one-iteration
calls (each of which bins synchronously): compared bitwise.  When the
primitives grow beyond the capacity, the refinement is rolled back to its
restart point and redone with larger buffers, with the same result.
"""
import numpy as np
import pytest

from oracle import field as F
from synth import fields as S

pytestmark = pytest.mark.gpu


def _lib():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    return g, torch


def _trajectories(g, torch, theta, field, grid, iters, lr, deterministic=True, **kw):
    ctx = g.Context(k=3.0, lr=lr, deterministic=deterministic, **kw)
    gg = g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0)
    ft = torch.from_numpy(field).cuda()
    a = g.Params(ctx, theta.shape[1]).upload(theta)
    la = g.refine(ctx, a, ft, gg, iters)
    resized = ctx.stats()["n_resized"]
    ctx2 = g.Context(k=3.0, lr=lr, deterministic=deterministic, **kw)
    b = g.Params(ctx2, theta.shape[1]).upload(theta)
    lb = np.concatenate([g.refine(ctx2, b, ft, gg, 1) for _ in range(iters)])
    return a.download(), la, b.download(), lb, resized, ctx


@pytest.mark.parametrize("shape", [(8, 32), (16, 16)])
def test_async_refine_equals_one_iteration_calls(shape):
    g, torch = _lib()
    f, _ = S.tiny_mixture(seed=3, normalize=True)
    grid = F.Grid(64, 64, 64)
    theta = S.random_params(2048, 64, seed=4, scale_range=(1.5, 4.0)).astype(np.float32)
    print(f"async refine 64^3 x 2048 shape {shape}", flush=True)
    ta, la, tb, lb, resized, ctx = _trajectories(g, torch, theta, f, grid, 8, 5e-3,
                                                 brick=shape[0], brick_z=shape[1])
    assert resized == 0
    assert np.array_equal(la, lb)
    assert np.array_equal(ta, tb)
    assert ctx.stats()["n_overlaps"] > 0


def test_capacity_overflow_rolls_back_to_the_same_result():
    """Primitives far narrower than a constant target grow by e^0.3 per step
    (Adam's first steps are lr sign(g)), so their box pairs outgrow the
    capacity sized at the first iteration: the refinement is redone."""
    g, torch = _lib()
    grid = F.Grid(96, 80, 72, 2, -1, 3)
    n = 3000
    theta = S.random_params(n, (96, 80, 72), seed=6, scale_range=(0.7, 1.0)).astype(np.float32)
    theta[0] += 2
    theta[1] -= 1
    theta[2] += 3
    theta[10] = 0.2
    field = np.ones(grid.shape, dtype=np.float32)
    print(f"async refine overflow {grid} x {n}", flush=True)
    ta, la, tb, lb, resized, ctx = _trajectories(g, torch, theta, field, grid, 6, 0.3, brick=8,
                                                 brick_z=8)
    assert resized == 1
    assert np.array_equal(la, lb)
    assert np.array_equal(ta, tb)
    # the redone refinement left the buffers large enough for the next one
    g.refine(ctx, g.Params(ctx, n).upload(ta.astype(np.float32)), torch.from_numpy(field).cuda(),
             g.Grid(96, 80, 72, 2, -1, 3), 2)


def test_atomic_async_refine_matches_oracle_trajectory():
    """Float-atomic sums: the asynchronous iterations follow the oracle's
    refinement (loss before each step within 1e-3)."""
    g, torch = _lib()
    grid = F.Grid(40, 36, 33, 1, 2, -3)
    theta = S.random_params(120, (40, 36, 33), seed=8, scale_range=(0.8, 3.0)).astype(np.float32)
    theta[0] += 1
    theta[1] += 2
    theta[2] -= 3
    field = np.random.default_rng(9).uniform(size=grid.shape).astype(np.float32)
    ctx = g.Context(k=3.0, lr=1e-2)
    p = g.Params(ctx, 120).upload(theta)
    got = g.refine(ctx, p, torch.from_numpy(field).cuda(), g.Grid(40, 36, 33, 1, 2, -3), 6)
    _, _, ref = F.refine(theta.astype(np.float64), field.astype(np.float64), grid, 3.0, 6, 1e-2)
    assert np.allclose(got, ref, rtol=1e-3)
