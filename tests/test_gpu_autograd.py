"""GPU check of the autograd bridge: the VJP of the truncated field against the
oracle's analytic gradient of a linear functional sum_p W(p) V(p)."""
import numpy as np
import pytest

from oracle import field as F
from synth import fields as S
from tests.parity import BAND, check_grad

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("deterministic", [True, False])
def test_autograd_vjp_matches_oracle(deterministic):
    import torch

    import paper_2608_14112_amd as g
    from paper_2608_14112_amd.autograd import GaussianField

    grid = F.Grid(29, 33, 26)
    params = S.random_params(35, (29, 33, 26), seed=2, scale_range=(0.8, 3.0), unit_quat=False)
    params = params.astype(np.float32).astype(np.float64)
    W = np.random.default_rng(3).normal(size=grid.shape).astype(np.float32)
    mod = GaussianField(35, g.Grid(29, 33, 26), k=3.0)
    mod.gctx.set_options(deterministic=1 if deterministic else 0)
    theta = torch.tensor(params.astype(np.float32), device="cuda", requires_grad=True)
    V = mod(theta)
    (V * torch.from_numpy(W).cuda()).sum().backward()
    got = theta.grad.cpu().numpy().astype(np.float64)
    # sum_p W dV/dtheta = gradient of sum (V - U)^2 with U = V_ref - W / 2
    Vr, _ = F.evaluate_windowed(params, grid, 3.0)
    U = Vr - 0.5 * W.astype(np.float64)
    _, ref = F.loss_grad(params, U, grid, 3.0)
    slack, _ = F.boundary_slack(params, U, grid, 3.0, BAND)
    check_grad(got, ref, slack=slack)
    # the forward value is the evaluator's
    assert np.max(np.abs(V.detach().cpu().numpy() - Vr)) < 1e-4


def test_vjp_of_residual_equals_loss_gradient():
    import torch

    import paper_2608_14112_amd as g

    grid = g.Grid(24, 20, 22)
    params = S.random_params(20, (24, 20, 22), seed=4, scale_range=(1.0, 3.0)).astype(np.float32)
    target = np.random.default_rng(5).uniform(size=grid.shape).astype(np.float32)
    ctx = g.Context(k=3.0)
    p = g.Params(ctx, 20).upload(params)
    V = torch.empty(grid.shape, device="cuda")
    g.evaluate(ctx, p, grid, V)
    tgt = torch.from_numpy(target).cuda()
    grad_l = torch.empty((11, 20), device="cuda")
    g.loss_grad(ctx, p, tgt, grid, grad_l)
    grad_v = g.vjp(ctx, p, (2.0 * (V - tgt)).contiguous(), grid)
    a, b = grad_l.cpu().numpy(), grad_v.cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(a))


def test_autograd_against_oracle_finite_differences():
    """d/dtheta of sum_p W(p) V(p) through the module vs central differences of
    the oracle's float64 field (no voxel within 1e-4 of the cut, so the
    truncation mask is constant over the stencil)."""
    import torch

    import paper_2608_14112_amd as g
    from paper_2608_14112_amd.autograd import GaussianField

    grid = F.Grid(14, 12, 13)
    params = S.random_params(4, (14, 12, 13), seed=8, scale_range=(1.0, 2.5), unit_quat=False)
    params = params.astype(np.float32).astype(np.float64)
    _, _, (_, _, namb) = F.evaluate_windowed(params, grid, 3.0, band=1e-4)
    assert namb == 0
    W = np.random.default_rng(9).normal(size=grid.shape)
    mod = GaussianField(4, g.Grid(14, 12, 13), k=3.0)
    theta = torch.tensor(params.astype(np.float32), device="cuda", requires_grad=True)
    (mod(theta) * torch.from_numpy(W.astype(np.float32)).cuda()).sum().backward()
    got = theta.grad.cpu().numpy().astype(np.float64)

    def functional(p):
        return float(np.sum(W * F.evaluate_windowed(p, grid, 3.0)[0]))

    for i in range(params.shape[1]):
        for j in range(11):
            h = 1e-6 * max(1.0, abs(params[j, i]))
            pp, pm = params.copy(), params.copy()
            pp[j, i] += h
            pm[j, i] -= h
            fd = (functional(pp) - functional(pm)) / (2 * h)
            scale = np.max(np.abs(got[:, i])) + 1e-6
            assert abs(got[j, i] - fd) <= 1e-3 * abs(fd) + 2e-4 * scale, (i, j, got[j, i], fd)
