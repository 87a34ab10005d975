"""A context gives back every device buffer it grew when it is destroyed.

Each cycle creates a context, runs the calls that grow the most kinds of
workspace buffer (binning with deterministic gradient slots, the dense
reference path's residual), and destroys it; the device's free memory must
not keep falling from cycle to cycle.
"""
import numpy as np
import pytest

from synth import fields as S

pytestmark = pytest.mark.gpu


def test_destroy_frees_the_workspace():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    n_side, n = 96, 3000
    grid = g.Grid(n_side, n_side, n_side)
    theta = S.random_params(n, n_side, seed=3, scale_range=(1.0, 3.0)).astype(np.float32)
    field = torch.rand((n_side, n_side, n_side), device="cuda", dtype=torch.float32)
    grad = torch.empty((11, n), device="cuda", dtype=torch.float32)

    def cycle():
        ctx = g.Context(deterministic=True)
        P = g.Params(ctx, n).upload(theta)
        g.loss_grad(ctx, P, field, grid, grad)
        g.dense_loss_grad(ctx, P, field, grid, grad)
        torch.cuda.synchronize()
        ws = ctx.stats()["workspace_bytes"]
        P.close()
        ctx.close()
        torch.cuda.synchronize()
        return ws

    ws = cycle()                      # first cycle: library and torch warm up
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        cycle()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"workspace {ws / 1e6:.1f} MB per context, free memory change "
          f"{(free1 - free0) / 1e6:.1f} MB over 5 cycles", flush=True)
    assert ws > 4 * n_side ** 3       # the dense residual alone is M floats
    # a leak of the workspace would lose 5 x ws
    assert free0 - free1 < ws
