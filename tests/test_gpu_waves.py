"""Several waves per brick (brick_waves 2 and 4 with 8 x 8 columns): the
waves split a brick's (primitive, brick) pairs and add their forward sums in
wave order, so the loss and gradient must still be the oracle's, the
deterministic mode must stay bitwise reproducible and schedule-independent,
and the vector-Jacobian product and refinement must follow the oracle."""
import numpy as np
import pytest

from oracle import field as F
from synth import fields as S
from tests.parity import BAND, check_grad

pytestmark = pytest.mark.gpu

WAVES = [(8, 8, 2), (8, 8, 4), (8, 16, 2), (8, 16, 4), (8, 32, 2), (8, 32, 4)]


def _lib():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    return g, torch


def _gg(g, grid):
    return g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0)


def _case(n, grid, seed, scale_range=(0.8, 3.5)):
    p = S.random_params(n, (grid.nx, grid.ny, grid.nz), seed=seed, scale_range=scale_range,
                        unit_quat=False)
    p[0] += grid.x0
    p[1] += grid.y0
    p[2] += grid.z0
    return p.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("deterministic", [True, False])
@pytest.mark.parametrize("shape", WAVES)
def test_loss_grad_with_split_waves_matches_oracle(shape, deterministic):
    g, torch = _lib()
    grid = F.Grid(30, 26, 45, 1, -3, 2)
    params = _case(70, grid, 31)
    field = np.random.default_rng(32).uniform(-0.3, 1.0, size=grid.shape).astype(np.float32)
    print(f"split waves {shape} det={deterministic}", flush=True)
    ctx = g.Context(k=3.0, brick=shape[0], brick_z=shape[1], brick_waves=shape[2],
                    deterministic=deterministic)
    p = g.Params(ctx, params.shape[1]).upload(params.astype(np.float32))
    grad = torch.empty((11, params.shape[1]), device="cuda")
    L = g.loss_grad(ctx, p, torch.from_numpy(field).cuda(), _gg(g, grid), grad)
    assert ctx.stats()["bin_waves"] == shape[2]
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, 3.0)
    assert abs(L - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(params, field, grid, 3.0, BAND)
    check_grad(grad.cpu().numpy().astype(np.float64), gr, slack=slack)


def test_split_waves_tiny_workload_and_vjp():
    """64^3 mixture, 2,048 primitives: loss and gradient at every split, and
    the VJP with an upstream of 2 (Vhat - V) equals the loss gradient."""
    g, torch = _lib()
    field, _ = S.tiny_mixture(seed=0)
    grid = F.Grid(64, 64, 64)
    params = S.random_params(2048, 64, seed=12, scale_range=(1.5, 4.0), weight_range=(-0.2, 0.2))
    params = params.astype(np.float32).astype(np.float64)
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, 3.0)
    slack, _ = F.boundary_slack(params, field, grid, 3.0, BAND)
    ft = torch.from_numpy(field).cuda()
    for shape in WAVES:
        print(f"tiny split {shape}", flush=True)
        ctx = g.Context(k=3.0, brick=shape[0], brick_z=shape[1], brick_waves=shape[2],
                        deterministic=True)
        p = g.Params(ctx, 2048).upload(params.astype(np.float32))
        grad = torch.empty((11, 2048), device="cuda")
        L = g.loss_grad(ctx, p, ft, g.Grid(64, 64, 64), grad)
        assert abs(L - Lr) <= 1e-5 * Lr
        check_grad(grad.cpu().numpy().astype(np.float64), gr, slack=slack)
        V = g.evaluate(ctx, p, g.Grid(64, 64, 64))
        up = (2.0 * (V - ft)).contiguous()
        gv = torch.empty((11, 2048), device="cuda")
        g.vjp(ctx, p, up, g.Grid(64, 64, 64), gv)
        check_grad(gv.cpu().numpy().astype(np.float64), gr, slack=slack)


def test_split_waves_deterministic_and_schedule_independent():
    """Deterministic sums: two runs bitwise equal, and the three schedules
    give bitwise the same refinement for a given split (4,352 bricks of 8^3,
    so the XCD chunks remap)."""
    g, torch = _lib()
    grid = F.Grid(136, 128, 128)
    params = _case(3000, grid, 41, scale_range=(0.8, 3.0))
    field = np.random.default_rng(42).uniform(size=grid.shape).astype(np.float32)
    ft = torch.from_numpy(field).cuda()
    for waves in (2, 4):
        results = []
        for sched in (0, 1, 2, 1):
            print(f"schedules waves={waves} sched={sched}", flush=True)
            ctx = g.Context(k=3.0, brick=8, brick_z=8, brick_waves=waves, schedule=sched,
                            deterministic=True, lr=5e-3)
            p = g.Params(ctx, 3000).upload(params.astype(np.float32))
            h = g.refine(ctx, p, ft, _gg(g, grid), 3)
            results.append((p.download(), h))
        for th, h in results[1:]:
            assert np.array_equal(th, results[0][0]) and np.array_equal(h, results[0][1])


def test_split_waves_refine_trajectory_matches_oracle():
    g, torch = _lib()
    grid = F.Grid(24, 24, 40)
    gen = S.random_params(12, (24, 24, 40), seed=21, scale_range=(1.5, 3.0))
    field = S.mixture_field(gen, grid.shape).astype(np.float32)
    start = gen.copy()
    start[0:3] += np.random.default_rng(1).normal(0, 0.5, size=(3, 12))
    start[10] *= 0.7
    start = start.astype(np.float32).astype(np.float64)
    ref_p, _, ref_l = F.refine(start, field.astype(np.float64), grid, 3.0, 20, lr=1e-2)
    for waves in (2, 4):
        ctx = g.Context(k=3.0, brick=8, brick_z=16, brick_waves=waves, lr=1e-2)
        p = g.Params(ctx, 12).upload(start.astype(np.float32))
        losses = g.refine(ctx, p, torch.from_numpy(field).cuda(), g.Grid(24, 24, 40), 20)
        assert np.max(np.abs(losses - ref_l) / ref_l) < 1e-3
        assert np.max(np.abs(p.download().astype(np.float64) - ref_p)) < 1e-3


def test_unsupported_split_is_refused():
    g, torch = _lib()
    with pytest.raises(g.GveError):
        g.Context(brick=16, brick_z=16, brick_waves=2)
    with pytest.raises(g.GveError):
        g.Context(brick=8, brick_z=32, brick_waves=3)
