"""GPU parity of evaluation, loss/gradient, Adam and refinement vs the oracle.

Every case calls the HIP path through the C ABI (the Python binding) and the
float64 oracle on the same seeded inputs; tolerances are those of
tests/parity.py.
"""
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


SHAPES = [(8, 8), (8, 16), (8, 32), (16, 16)]


def _eval_gpu(g, torch, params, grid, k, brick):
    bxy, bz = brick if isinstance(brick, tuple) else (brick, brick)
    ctx = g.Context(k=k, brick=bxy, brick_z=bz)
    p = g.Params(ctx, params.shape[1]).upload(params.astype(np.float32))
    out = torch.empty(grid.shape, device="cuda", dtype=torch.float32)
    g.evaluate(ctx, p, g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0), out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ctx.stats()


def _case(n, grid, seed, scale_range=(0.6, 4.0)):
    p = S.random_params(n, (grid.nx, grid.ny, grid.nz), seed=seed, scale_range=scale_range,
                        unit_quat=False)
    # let some primitives hang over the grid faces
    p[0] += grid.x0 + np.random.default_rng(seed).uniform(-3, 3, n)
    p[1] += grid.y0
    p[2] += grid.z0
    return p.astype(np.float32).astype(np.float64)


CASES = [
    # (grid, n, seed): several bricks per axis with ragged tails, non-zero origins
    (F.Grid(37, 29, 21, 3, -2, 5), 60, 0),
    (F.Grid(17, 40, 33, -7, 0, 2), 45, 1),
]


@pytest.mark.parametrize("k", [3.0, 5.0])
@pytest.mark.parametrize("brick", SHAPES)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_evaluate_matches_oracle(k, brick, case):
    g, torch = _lib()
    grid, n, seed = CASES[case]
    print(f"evaluate grid={grid} n={n} seed={seed} k={k} B={brick}", flush=True)
    params = _case(n, grid, seed)
    got, st = _eval_gpu(g, torch, params, grid, k, brick)
    V, A, br = F.evaluate_windowed(params, grid, k, band=BAND)
    check_field(got, V, A, br)
    assert st["n_primitives"] == n and st["n_overlaps"] > 0
    # pair lists and sort buffers at least
    assert st["workspace_bytes"] >= 4 * 4 * st["n_overlaps"]


def test_evaluate_tiny_workload_size():
    """64^3 grid, 2,048 primitives with scales 1.5-4 (the small workload's budget)."""
    g, torch = _lib()
    grid = F.Grid(64, 64, 64)
    params = S.random_params(2048, 64, seed=7, scale_range=(1.5, 4.0)).astype(np.float32)
    params = params.astype(np.float64)
    print("evaluate 64^3 x 2048", flush=True)
    got, _ = _eval_gpu(g, torch, params, grid, 3.0, 8)
    V, A, br = F.evaluate_windowed(params, grid, 3.0, band=BAND)
    check_field(got, V, A, br)


def test_forward_is_bitwise_reproducible_and_brick_invariant():
    g, torch = _lib()
    grid = F.Grid(40, 33, 27)
    params = _case(80, grid, 3)
    a, _ = _eval_gpu(g, torch, params, grid, 3.0, 8)
    b, _ = _eval_gpu(g, torch, params, grid, 3.0, 8)
    assert np.array_equal(a, b)
    _, A = F.evaluate_windowed(params, grid, 3.0)
    # another brick shape changes only the float32 rounding of each column's
    # coordinates (both results are within 1e-5 A of the oracle)
    for shape in SHAPES[1:]:
        c, _ = _eval_gpu(g, torch, params, grid, 3.0, shape)
        assert np.max(np.abs(a.astype(np.float64) - c) / (A + 1e-30)) < 1e-5


def _support_bricks(params, grid, k, bxy, bz):
    """(primitive, brick) pairs whose brick holds a voxel with m^2 < k^2 (1 + 1e-4),
    and pairs whose brick meets the primitive's k-sigma box (float64 definitions)."""
    cov = F.covariance(params)
    P = F.precision(params)
    mu = params[0:3].T
    nsup = nbox = 0
    for i in range(params.shape[1]):
        box = F.support_box(mu[i], cov[i], k, grid)
        if box is None:
            continue
        (ia, ib), (ja, jb), (ka, kb) = box
        nbox += (ib // bxy - ia // bxy + 1) * (jb // bxy - ja // bxy + 1) * (kb // bz - ka // bz + 1)
        dx, dy, dz = F._box_offsets(box, mu[i], grid)
        inside = F._quad(P[i], dx, dy, dz) < k * k * (1 + 1e-4)
        zz, yy, xx = np.nonzero(inside)
        keys = {((x + ia) // bxy, (y + ja) // bxy, (z + ka) // bz) for x, y, z in zip(xx, yy, zz)}
        nsup += len(keys)
    return nsup, nbox


@pytest.mark.parametrize("brick", [(8, 32), (16, 16)])
def test_brick_culling_keeps_every_brick_with_support(brick):
    """Binning drops bricks a separating plane parts from the support, in
    both gradient modes.  The field is bitwise the same in both, and the kept
    pairs lie between the bricks that hold support and the bricks of the box."""
    g, torch = _lib()
    grid = F.Grid(48, 44, 70, 2, -1, 3)
    rng = np.random.default_rng(21)
    p = S.random_params(120, (48, 44, 70), seed=21, scale_range=(0.7, 2.0), unit_quat=False)
    p[7] += rng.uniform(0.5, 1.6, p.shape[1])          # elongated: log-scale spread up to ~5x
    p[0] += grid.x0
    p[1] += grid.y0
    p[2] += grid.z0
    p = p.astype(np.float32).astype(np.float64)
    bxy, bz = brick
    outs, pairs = [], []
    for det in (False, True):
        ctx = g.Context(k=3.0, brick=bxy, brick_z=bz, deterministic=det)
        P = g.Params(ctx, p.shape[1]).upload(p.astype(np.float32))
        out = torch.empty(grid.shape, device="cuda", dtype=torch.float32)
        g.evaluate(ctx, P, g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0), out)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        pairs.append(ctx.stats()["n_overlaps"])
    assert np.array_equal(outs[0], outs[1])
    assert pairs[0] == pairs[1]
    nsup, nbox = _support_bricks(p, grid, 3.0, bxy, bz)
    print(f"support {nsup}, kept {pairs[0]}, box {nbox}", flush=True)
    assert nsup <= pairs[0] < 0.95 * nbox
    V, A, br = F.evaluate_windowed(p, grid, 3.0, band=BAND)
    check_field(outs[0], V, A, br)


def test_large_k_equals_untruncated_field():
    g, torch = _lib()
    grid = F.Grid(30, 30, 30)
    params = _case(20, grid, 4, scale_range=(0.8, 2.0))
    got, _ = _eval_gpu(g, torch, params, grid, 8.0, 8)
    ref = F.evaluate_bruteforce(params, grid, None)
    _, A = F.evaluate_windowed(params, grid, 8.0)
    check_field(got, ref, A)


def test_edge_cases():
    g, torch = _lib()
    # every primitive outside the grid: no pairs, zero field
    grid = F.Grid(12, 12, 12)
    p = _case(10, grid, 5, scale_range=(0.5, 1.0))
    p[0] += 100.0
    got, st = _eval_gpu(g, torch, p, grid, 3.0, 8)
    assert st["n_overlaps"] == 0 and not np.any(got)
    # a single voxel
    grid1 = F.Grid(1, 1, 1, 5, 5, 5)
    p1 = _case(4, F.Grid(3, 3, 3, 4, 4, 4), 6, scale_range=(0.7, 2.0))
    got1, _ = _eval_gpu(g, torch, p1, grid1, 3.0, 8)
    V1, A1 = F.evaluate_windowed(p1, grid1, 3.0)
    check_field(got1, V1, A1)
    # zero quaternion is the identity rotation
    grid2 = F.Grid(9, 8, 17)
    p2 = _case(6, grid2, 8)
    p2[3:7, 0] = 0.0
    p2[3:7, 3] = 1e-14                       # |q| = 2e-14: also below the limit
    got2, st2 = _eval_gpu(g, torch, p2, grid2, 3.0, 16)
    V2, A2, br = F.evaluate_windowed(p2, grid2, 3.0, band=BAND)
    check_field(got2, V2, A2, br)
    assert st2["n_degenerate_q"] == 2        # counted


# ----------------------------------------------------------------------------- gradient

def _loss_grad_gpu(g, torch, params, field, grid, k, brick, deterministic=True):
    bxy, bz = brick if isinstance(brick, tuple) else (brick, brick)
    ctx = g.Context(k=k, brick=bxy, brick_z=bz, deterministic=deterministic)
    p = g.Params(ctx, params.shape[1]).upload(params.astype(np.float32))
    f = torch.from_numpy(np.ascontiguousarray(field, dtype=np.float32)).cuda()
    grad = torch.empty((11, params.shape[1]), device="cuda", dtype=torch.float32)
    L = g.loss_grad(ctx, p, f, g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0), grad)
    return L, grad.cpu().numpy()


@pytest.mark.parametrize("deterministic", [True, False])
@pytest.mark.parametrize("brick", SHAPES)
@pytest.mark.parametrize("k", [3.0, 5.0])
def test_loss_grad_matches_oracle(brick, k, deterministic):
    g, torch = _lib()
    grid = F.Grid(30, 26, 22, 1, -3, 2)
    params = _case(40, grid, 10, scale_range=(0.8, 3.5))
    field = np.random.default_rng(11).uniform(-0.3, 1.0, size=grid.shape).astype(np.float32)
    print(f"loss_grad k={k} B={brick} det={deterministic}", flush=True)
    L, grad = _loss_grad_gpu(g, torch, params, field, grid, k, brick, deterministic)
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, k)
    assert abs(L - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(params, field, grid, k, BAND)
    check_grad(grad, gr, slack=slack)


def test_loss_grad_edge_cases():
    """Gradient edge cases: every primitive outside the grid (no pairs: zero
    gradient, L = sum V^2), a single primitive, and a zero quaternion (the
    identity rotation; its quaternion gradient is zero), on grids thinner than
    one brick in z."""
    g, torch = _lib()
    grid = F.Grid(13, 11, 5, 2, -1, 0)
    field = np.random.default_rng(17).uniform(-0.5, 1.0, size=grid.shape).astype(np.float32)
    p = _case(8, grid, 18, scale_range=(0.5, 1.5))
    p[0] += 200.0
    for det in (True, False):
        L, grad = _loss_grad_gpu(g, torch, p, field, grid, 3.0, (8, 32), deterministic=det)
        assert not np.any(grad)
        assert abs(L - np.sum(field.astype(np.float64) ** 2)) <= 1e-6 * L
    # refinement and the vector-Jacobian product with no pairs: zero gradient,
    # parameters unchanged, every loss sum V^2
    gg = g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0)
    f = torch.from_numpy(field).cuda()
    for det in (True, False):
        ctx = g.Context(k=3.0, deterministic=det)
        P = g.Params(ctx, p.shape[1]).upload(p.astype(np.float32))
        hist = g.refine(ctx, P, f, gg, 3)
        assert np.allclose(hist, np.sum(field.astype(np.float64) ** 2), rtol=1e-6)
        assert np.array_equal(P.download(), p.astype(np.float32))
        assert not np.any(g.vjp(ctx, P, f, gg).cpu().numpy())
    p1 = _case(1, grid, 19, scale_range=(1.0, 2.0))
    L1, g1 = _loss_grad_gpu(g, torch, p1, field, grid, 3.0, (8, 32))
    Lr1, gr1 = F.loss_grad(p1, field.astype(np.float64), grid, 3.0)
    assert abs(L1 - Lr1) <= 1e-5 * Lr1
    slack1, _ = F.boundary_slack(p1, field, grid, 3.0, BAND)
    check_grad(g1, gr1, slack=slack1)
    p2 = _case(6, grid, 20, scale_range=(0.8, 2.0))
    p2[3:7, 0] = 0.0
    L2, g2 = _loss_grad_gpu(g, torch, p2, field, grid, 3.0, (8, 8))
    Lr2, gr2 = F.loss_grad(p2, field.astype(np.float64), grid, 3.0)
    assert abs(L2 - Lr2) <= 1e-5 * Lr2
    assert np.all(g2[3:7, 0] == 0.0) and np.all(gr2[3:7, 0] == 0.0)
    slack2, _ = F.boundary_slack(p2, field, grid, 3.0, BAND)
    check_grad(g2, gr2, slack=slack2)


@pytest.mark.parametrize("kind", ["wide", "thin"])
def test_loss_grad_both_backward_forms(kind):
    """The backward pass evaluates G along each column by a product recurrence
    when a pair's recorded span times s_z is short enough, else directly.
    Wide primitives (sigma 2.5-5, s_z about 0.2) take the recurrence; primitives
    thin in one axis (0.35-0.6, rotated, s_z up to about 2.4) take the direct form
    for most pairs.  Both against the oracle, atomic sums, 8x8x32 bricks."""
    g, torch = _lib()
    grid = F.Grid(40, 36, 70, 2, 0, -5)
    rng = np.random.default_rng(31 if kind == "wide" else 32)
    n = 50
    p = S.random_params(n, (40, 36, 70), seed=33, scale_range=(2.5, 5.0), unit_quat=False)
    if kind == "thin":
        p[9] = np.log(rng.uniform(0.35, 0.6, n))
    p[0] += grid.x0
    p[1] += grid.y0
    p[2] += grid.z0
    p = p.astype(np.float32).astype(np.float64)
    field = rng.uniform(-0.2, 1.0, size=grid.shape).astype(np.float32)
    L, grad = _loss_grad_gpu(g, torch, p, field, grid, 3.0, (8, 32), deterministic=False)
    Lr, gr = F.loss_grad(p, field.astype(np.float64), grid, 3.0)
    assert abs(L - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(p, field, grid, 3.0, BAND)
    check_grad(grad, gr, slack=slack)


@pytest.mark.parametrize("waves", [1, 2])
@pytest.mark.parametrize("deterministic", [True, False])
def test_loss_grad_crowded_bricks(deterministic, waves):
    """1,500 primitives in a 16 x 16 x 32 grid: each of its four 8 x 8 x 32
    bricks holds well over the 512 pairs whose active offsets the forward
    pass records, so the backward pass also runs its unrecorded form (the
    box z-range with a support test per offset) for the later pairs."""
    g, torch = _lib()
    grid = F.Grid(16, 16, 32, 0, 0, 0)
    n = 1500
    p = S.random_params(n, (16, 16, 32), seed=61, scale_range=(1.0, 3.0),
                        weight_range=(-0.2, 0.2), unit_quat=False)
    p = p.astype(np.float32).astype(np.float64)
    field = np.random.default_rng(62).uniform(-0.5, 1.0, size=grid.shape).astype(np.float32)
    ctx = g.Context(k=3.0, brick=8, brick_z=32, brick_waves=waves, deterministic=deterministic)
    pp = g.Params(ctx, n).upload(p.astype(np.float32))
    f = torch.from_numpy(field).cuda()
    grad = torch.empty((11, n), device="cuda", dtype=torch.float32)
    L = g.loss_grad(ctx, pp, f, g.Grid(16, 16, 32), grad)
    pairs = ctx.stats()["n_overlaps"]
    print(f"crowded bricks: {pairs} pairs over 4 bricks", flush=True)
    assert pairs > 4 * 600  # > 512 per brick on average
    Lr, gr = F.loss_grad(p, field.astype(np.float64), grid, 3.0)
    assert abs(L - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(p, field, grid, 3.0, BAND)
    check_grad(grad.cpu().numpy().astype(np.float64), gr, slack=slack)


def test_deterministic_gradient_is_bitwise_reproducible():
    g, torch = _lib()
    grid = F.Grid(40, 36, 44)
    params = _case(120, grid, 13, scale_range=(0.8, 4.0))
    field = np.random.default_rng(14).uniform(size=grid.shape).astype(np.float32)
    L1, g1 = _loss_grad_gpu(g, torch, params, field, grid, 3.0, (8, 32), True)
    L2, g2 = _loss_grad_gpu(g, torch, params, field, grid, 3.0, (8, 32), True)
    assert L1 == L2 and np.array_equal(g1, g2)


def test_loss_grad_tiny_workload():
    """64^3 signed-mixture target, 2,048 primitives, k = 3."""
    g, torch = _lib()
    field, _ = S.tiny_mixture(seed=0)
    grid = F.Grid(64, 64, 64)
    params = S.random_params(2048, 64, seed=12, scale_range=(1.5, 4.0), weight_range=(-0.2, 0.2))
    params = params.astype(np.float32).astype(np.float64)
    Lr, gr = F.loss_grad(params, field.astype(np.float64), grid, 3.0)
    slack, _ = F.boundary_slack(params, field, grid, 3.0, BAND)
    for shape in ((8, 8), (8, 16), (8, 32), (16, 16)):
        L, grad = _loss_grad_gpu(g, torch, params, field, grid, 3.0, shape)
        assert abs(L - Lr) <= 1e-5 * Lr
        check_grad(grad, gr, slack=slack)


def test_adam_step_matches_oracle():
    g, torch = _lib()
    rng = np.random.default_rng(0)
    n = 1000
    theta = rng.normal(size=(11, n)).astype(np.float32)
    ctx = g.Context(lr=3e-3, ell_min=-1.0, ell_max=1.5)
    p = g.Params(ctx, n).upload(theta)
    st = F.AdamState.zeros(n)
    ref = theta.astype(np.float64)
    for it in range(3):
        gr = rng.normal(size=(11, n)).astype(np.float32)
        g.adam_step(ctx, p, torch.from_numpy(gr).cuda())
        ref, _ = F.adam_update(ref, gr.astype(np.float64), st, lr=3e-3, ell_clamp=(-1.0, 1.5))
    got = p.download().astype(np.float64)
    assert p.step == 3
    assert np.max(np.abs(got - ref)) < 1e-6 * (1 + np.max(np.abs(ref)))


@pytest.mark.parametrize("deterministic", [True, False])
def test_refine_trajectory_matches_oracle(deterministic):
    g, torch = _lib()
    grid = F.Grid(24, 24, 24)
    gen = S.random_params(12, 24, seed=21, scale_range=(1.5, 3.0))
    field = S.mixture_field(gen, grid.shape).astype(np.float32)
    start = gen.copy()
    start[0:3] += np.random.default_rng(1).normal(0, 0.5, size=(3, 12))
    start[10] *= 0.7
    start = start.astype(np.float32).astype(np.float64)
    ctx = g.Context(k=3.0, brick=8, lr=1e-2, deterministic=deterministic)
    p = g.Params(ctx, 12).upload(start.astype(np.float32))
    f = torch.from_numpy(field).cuda()
    losses = g.refine(ctx, p, f, g.Grid(24, 24, 24), 20)
    ref_p, _, ref_l = F.refine(start, field.astype(np.float64), grid, 3.0, 20, lr=1e-2)
    rel = np.abs(losses - ref_l) / ref_l
    assert np.max(rel) < 1e-3, rel
    got = p.download().astype(np.float64)
    assert np.max(np.abs(got - ref_p)) < 1e-3
    assert p.step == 20 and losses[-1] < losses[0]


@pytest.mark.parametrize("deterministic", [True, False])
def test_refine_reports_non_finite_parameters_without_a_loss_history(deterministic):
    """A NaN weight planted from the host spreads through the residual to the
    gradients of every primitive it overlaps; the update counts the parameters
    it leaves non-finite and gve_refine returns NUMERIC even when no loss
    history is requested.  (The kernels take NaN arithmetic without faults: a
    NaN in mu or a scale gives an empty box, a NaN weight changes only values.)"""
    g, torch = _lib()
    grid = F.Grid(40, 36, 33)
    params = _case(80, grid, 4).astype(np.float32)
    params[10, 5] = np.nan
    field = np.random.default_rng(3).uniform(size=grid.shape).astype(np.float32)
    ctx = g.Context(k=3.0, deterministic=deterministic)
    p = g.Params(ctx, 80).upload(params)
    gg = g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0)
    assert ctx.stats()["n_nonfinite"] == 0
    with pytest.raises(g.GveError) as e:
        g.refine(ctx, p, torch.from_numpy(field).cuda(), gg, 2, want_losses=False)
    assert e.value.status == g.NUMERIC
    st = ctx.stats()
    assert st["n_nonfinite"] > 0
    # counted per step: at least the entries non-finite now
    assert np.count_nonzero(~np.isfinite(p.download())) <= st["n_nonfinite"]
    # a finite set on the same context refines without the error
    q = g.Params(ctx, 80).upload(np.nan_to_num(params, nan=0.1))
    g.refine(ctx, q, torch.from_numpy(field).cuda(), gg, 2, want_losses=False)
    assert ctx.stats()["n_nonfinite"] == st["n_nonfinite"]


def test_count_pairs_fills_the_work_counters():
    g, torch = _lib()
    grid = F.Grid(37, 29, 21, 3, -2, 5)
    params = _case(60, grid, 0)
    ctx = g.Context(k=3.0)
    p = g.Params(ctx, 60).upload(params.astype(np.float32))
    nin, ncand = g.count_pairs(ctx, p, g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0,
                                              grid.z0))
    st = ctx.stats()
    assert st["n_in_support"] == nin and st["n_candidates"] == ncand
    assert 0 < st["n_atomics"] <= st["n_overlaps"]
    assert nin <= ncand <= 64 * 32 * st["n_atomics"]
