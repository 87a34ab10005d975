"""GPU parity of the dense reference path (every (primitive, voxel) pair
evaluated, no bricks) against the oracle, and its agreement with the binned
path on the same inputs.

The dense path is the baseline that truncation-aware binning is timed against
(Sec. III-G), so it must compute the same truncated field, loss and gradient.
Cases cover ragged rows (nx not a multiple of 64), primitive counts that are
not multiples of 64, non-zero origins, primitives hanging over or lying
outside the grid, and one-voxel rows.
"""
import ctypes

import numpy as np
import pytest

from oracle import field as F
from synth import fields as S
from tests.parity import BAND, check_field, check_grad

pytestmark = pytest.mark.gpu


def _lib():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return g, torch


def _case(n, grid, seed, scale_range=(0.6, 4.0)):
    p = S.random_params(n, (grid.nx, grid.ny, grid.nz), seed=seed, scale_range=scale_range,
                        unit_quat=False)
    p[0] += grid.x0 + np.random.default_rng(seed).uniform(-3, 3, n)
    p[1] += grid.y0
    p[2] += grid.z0
    return p.astype(np.float32).astype(np.float64)


def _ggrid(g, grid):
    return g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0)


def _dense_eval(g, torch, params, grid, k):
    ctx = g.Context(k=k)
    p = g.Params(ctx, params.shape[1]).upload(params.astype(np.float32))
    out = g.dense_evaluate(ctx, p, _ggrid(g, grid))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _dense_loss_grad(g, torch, params, field, grid, k):
    ctx = g.Context(k=k)
    p = g.Params(ctx, params.shape[1]).upload(params.astype(np.float32))
    f = torch.from_numpy(np.ascontiguousarray(field, dtype=np.float32)).cuda()
    grad = torch.empty((11, params.shape[1]), device="cuda", dtype=torch.float32)
    L = g.dense_loss_grad(ctx, p, f, _ggrid(g, grid), grad)
    return L, grad.cpu().numpy()


CASES = [
    (F.Grid(37, 29, 21, 3, -2, 5), 70, 0),
    (F.Grid(17, 40, 33, -7, 0, 2), 130, 1),
    (F.Grid(1, 23, 19, 4, 1, -3), 9, 2),      # one-voxel rows
]


@pytest.mark.parametrize("k", [3.0, 5.0])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_dense_evaluate_matches_oracle(k, case):
    g, torch = _lib()
    grid, n, seed = CASES[case]
    print(f"dense evaluate grid={grid} n={n} k={k}", flush=True)
    params = _case(n, grid, seed)
    got = _dense_eval(g, torch, params, grid, k)
    V, A, br = F.evaluate_windowed(params, grid, k, band=BAND)
    check_field(got, V, A, br)


@pytest.mark.parametrize("k", [3.0, 5.0])
def test_dense_loss_grad_matches_oracle(k):
    g, torch = _lib()
    grid = F.Grid(30, 26, 22, 1, -3, 2)
    params = _case(70, grid, 10, scale_range=(0.8, 3.5))
    field = np.random.default_rng(11).uniform(-0.3, 1.0, size=grid.shape).astype(np.float32)
    print(f"dense loss_grad k={k}", flush=True)
    L, grad = _dense_loss_grad(g, torch, params, field, grid, k)
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, k)
    assert abs(L - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(params, field, grid, k, BAND)
    check_grad(grad, gr, slack=slack)


def test_dense_and_binned_agree_on_the_small_workload():
    """64^3 signed-mixture target, 2,048 primitives, k = 3: dense and binned
    fields and gradients both meet the oracle's tolerance.  (They are not
    compared with each other directly: the two compute m^2 with different
    float32 roundings, so a pair lying on the cut may be kept by one and
    dropped by the other, which the oracle's bracket allows.)"""
    g, torch = _lib()
    field, _ = S.tiny_mixture(seed=0)
    grid = F.Grid(64, 64, 64)
    params = S.random_params(2048, 64, seed=12, scale_range=(1.5, 4.0), weight_range=(-0.2, 0.2))
    params = params.astype(np.float32).astype(np.float64)
    print("dense vs binned 64^3 x 2048", flush=True)
    ctx = g.Context(k=3.0)
    P = g.Params(ctx, 2048).upload(params.astype(np.float32))
    gg = _ggrid(g, grid)
    vd = g.dense_evaluate(ctx, P, gg).cpu().numpy()
    vb = g.evaluate(ctx, P, gg).cpu().numpy()
    V, A, br = F.evaluate_windowed(params, grid, 3.0, band=BAND)
    check_field(vd, V, A, br)
    check_field(vb, V, A, br)
    f = torch.from_numpy(np.ascontiguousarray(field, dtype=np.float32)).cuda()
    gd = torch.empty((11, 2048), device="cuda", dtype=torch.float32)
    gb = torch.empty_like(gd)
    Ld = g.dense_loss_grad(ctx, P, f, gg, gd)
    Lb = g.loss_grad(ctx, P, f, gg, gb)
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, 3.0)
    assert abs(Ld - Lr) <= 1e-5 * Lr and abs(Lb - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(params, field, grid, 3.0, BAND)
    check_grad(gd.cpu().numpy(), gr, slack=slack)
    check_grad(gb.cpu().numpy(), gr, slack=slack)


def test_dense_primitives_outside_the_grid_add_nothing():
    """A primitive whose support lies outside the grid contributes no value
    and gets a zero gradient; the others are unaffected."""
    g, torch = _lib()
    grid = F.Grid(20, 18, 16)
    params = _case(5, grid, 4, scale_range=(1.0, 2.0))
    params[0:3, 2] = (200.0, -150.0, 90.0)
    field = np.random.default_rng(5).uniform(size=grid.shape).astype(np.float32)
    L, grad = _dense_loss_grad(g, torch, params, field, grid, 3.0)
    assert np.all(grad[:, 2] == 0.0)
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, 3.0)
    assert abs(L - Lr) <= 1e-5 * Lr
    check_grad(grad, gr)


def test_dense_argument_errors():
    g, torch = _lib()
    ctx = g.Context()
    P = g.Params(ctx, 4).upload(S.random_params(4, 8, seed=0).astype(np.float32))
    gg = g.Grid(8, 8, 8)
    assert g._lib.gve_dense_evaluate(ctx.handle, P.handle, gg.c(), None) != 0
    assert g._lib.gve_dense_loss_grad(ctx.handle, P.handle, None, gg.c(), None,
                                      ctypes.byref(ctypes.c_double())) != 0
    with pytest.raises(g.GveError):
        g.dense_evaluate(ctx, P, g.Grid(0, 8, 8))
