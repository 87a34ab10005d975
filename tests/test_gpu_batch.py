"""GPU checks of batched volumes, brick schedules and the autotuner.

A batch is several uneven volumes (different sizes, origins, primitive
counts) binned and refined together.  Each volume's work in a batch is the
work of a separate call, so batch results must equal per-volume calls bitwise
(deterministic gradient sums) and match the oracle volume by volume; every
schedule (brick order, XCD-grouped order, persistent heaviest-first queue)
must give bitwise the same results.
"""
import numpy as np
import pytest

from oracle import field as F
from synth import fields as S
from tests.parity import BAND, check_field, check_grad

pytestmark = pytest.mark.gpu

VOLUMES = [  # (grid, primitives, seed): ragged against every brick shape, mixed origins
    (F.Grid(37, 29, 21, 3, -2, 5), 60, 0),
    (F.Grid(5, 3, 2, 0, 0, 0), 4, 1),           # smaller than one brick
    (F.Grid(17, 40, 33, -7, 0, 2), 45, 2),
    (F.Grid(24, 24, 24, 100, 50, -30), 70, 3),
    (F.Grid(9, 31, 47, 0, 0, 0), 25, 4),
]


def _lib():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    return g, torch


def _params(grid, n, seed):
    p = S.random_params(n, (grid.nx, grid.ny, grid.nz), seed=seed, scale_range=(0.6, 4.0),
                        unit_quat=False)
    p[0] += grid.x0 + np.random.default_rng(seed).uniform(-3, 3, n)
    p[1] += grid.y0
    p[2] += grid.z0
    if seed == 3:
        p[0, :3] += 500.0           # primitives whose box misses their volume
    return p.astype(np.float32).astype(np.float64)


def _field(grid, seed):
    gen = S.random_params(12, (grid.nx, grid.ny, grid.nz), seed=100 + seed,
                          scale_range=(1.0, 4.0))
    return S.mixture_field(gen, grid.shape).astype(np.float32)


def _ggrid(g, grid):
    return g.Grid(grid.nx, grid.ny, grid.nz, grid.x0, grid.y0, grid.z0)


def _setup(g, torch, vols=VOLUMES, **ctx_kw):
    ctx_kw.setdefault("deterministic", True)      # bitwise comparisons below
    ctx = g.Context(k=3.0, lr=5e-3, **ctx_kw)
    B = g.Batch(ctx, [_ggrid(g, v[0]) for v in vols], [v[1] for v in vols])
    thetas = [_params(*v) for v in vols]
    fields = [_field(v[0], v[2]) for v in vols]
    for i, th in enumerate(thetas):
        B.set_item(i, g.Params(ctx, th.shape[1]).upload(th.astype(np.float32)))
    cat = torch.from_numpy(np.concatenate([f.ravel() for f in fields])).cuda()
    return ctx, B, thetas, fields, cat


def test_offsets_and_items_roundtrip():
    g, torch = _lib()
    ctx, B, thetas, fields, cat = _setup(g, torch)
    assert list(B.prim_offsets) == list(np.cumsum([0] + [v[1] for v in VOLUMES]))
    assert B.voxel_offsets[-1] == sum(v[0].nx * v[0].ny * v[0].nz for v in VOLUMES)
    full = B.params.download()
    for i, th in enumerate(thetas):
        a, b = B.prim_offsets[i], B.prim_offsets[i + 1]
        assert np.array_equal(full[:, a:b], th.astype(np.float32))
        q = B.get_item(i, g.Params(ctx, th.shape[1]))
        assert np.array_equal(q.download(), th.astype(np.float32))
    with pytest.raises(g.GveError):
        B.set_item(0, g.Params(ctx, 3))
    with pytest.raises(g.GveError):
        B.set_item(len(VOLUMES), g.Params(ctx, 3))


@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_batch_matches_oracle_per_volume(schedule):
    g, torch = _lib()
    ctx, B, thetas, fields, cat = _setup(g, torch, schedule=schedule)
    out = g.batch_evaluate(ctx, B).cpu().numpy()
    grad = torch.empty((11, B.params.n), device="cuda")
    losses = g.batch_loss_grad(ctx, B, cat, grad)
    grad = grad.cpu().numpy().astype(np.float64)
    for i, (grid, n, seed) in enumerate(VOLUMES):
        a, b = B.voxel_offsets[i], B.voxel_offsets[i + 1]
        V, A, bracket = F.evaluate_windowed(thetas[i], grid, 3.0, band=BAND)
        check_field(out[a:b].reshape(grid.shape), V, A, bracket)
        Lr, gr = F.loss_grad(thetas[i], fields[i].astype(np.float64), grid, 3.0)
        assert abs(losses[i] - Lr) <= 1e-5 * max(Lr, 1e-12), (i, losses[i], Lr)
        pa, pb = B.prim_offsets[i], B.prim_offsets[i + 1]
        slack, _ = F.boundary_slack(thetas[i], fields[i], grid, 3.0, BAND)
        check_grad(grad[:, pa:pb], gr, slack=slack)


def test_batch_equals_separate_calls_bitwise():
    g, torch = _lib()
    ctx, B, thetas, fields, cat = _setup(g, torch)
    out = g.batch_evaluate(ctx, B).cpu().numpy()
    grad = torch.empty((11, B.params.n), device="cuda")
    g.batch_loss_grad(ctx, B, cat, grad)
    grad = grad.cpu().numpy()
    hist = g.batch_refine(ctx, B, cat, 6)
    after = B.params.download()
    for i, (grid, n, seed) in enumerate(VOLUMES):
        gg = _ggrid(g, grid)
        p = g.Params(ctx, n).upload(thetas[i].astype(np.float32))
        a, b = B.voxel_offsets[i], B.voxel_offsets[i + 1]
        assert np.array_equal(g.evaluate(ctx, p, gg).cpu().numpy().ravel(), out[a:b])
        gi = torch.empty((11, n), device="cuda")
        g.loss_grad(ctx, p, torch.from_numpy(fields[i]).cuda(), gg, gi)
        pa, pb = B.prim_offsets[i], B.prim_offsets[i + 1]
        assert np.array_equal(gi.cpu().numpy(), grad[:, pa:pb])
        hi = g.refine(ctx, p, torch.from_numpy(fields[i]).cuda(), gg, 6)
        assert np.array_equal(p.download(), after[:, pa:pb])
        assert np.allclose(hi, hist[:, i], rtol=1e-12, atol=0)


def test_schedules_give_identical_refinement():
    g, torch = _lib()
    results = []
    for sched in (0, 1, 2):
        for shape in ((8, 8), (16, 16)):
            ctx, B, thetas, fields, cat = _setup(g, torch, schedule=sched, brick=shape[0],
                                                 brick_z=shape[1])
            h = g.batch_refine(ctx, B, cat, 4)
            results.append((sched, shape, B.params.download(), h))
    for sched, shape, th, h in results:
        same = [r for r in results if r[1] == shape]
        assert np.array_equal(th, same[0][2]), (sched, shape)
        assert np.array_equal(h, same[0][3]), (sched, shape)


def test_batch_of_one_matches_single_volume():
    g, torch = _lib()
    grid, n, seed = VOLUMES[0]
    ctx, B, thetas, fields, cat = _setup(g, torch, vols=[VOLUMES[0]])
    h = g.batch_refine(ctx, B, cat, 3)
    p = g.Params(ctx, n).upload(thetas[0].astype(np.float32))
    hs = g.refine(ctx, p, torch.from_numpy(fields[0]).cuda(), _ggrid(g, grid), 3)
    assert np.array_equal(p.download(), B.params.download())
    assert np.array_equal(hs, h[:, 0])


def test_autotune_picks_a_candidate_and_caches():
    g, torch = _lib()
    ctx, B, thetas, fields, cat = _setup(g, torch)
    before = B.params.download()
    table = g.autotune(ctx, cat, batch=B, reps=2)
    assert len(table) == 30
    assert {(t[0], t[1], t[4]) for t in table} == {
        (8, 8, 1), (8, 8, 2), (8, 8, 4), (8, 16, 1), (8, 16, 2), (8, 16, 4), (8, 32, 1),
        (8, 32, 2), (8, 32, 4), (16, 16, 1)}
    assert all(t[3] > 0 for t in table)
    best = min(table, key=lambda t: t[3])
    o = ctx.options
    assert (o.brick, o.brick_z, o.schedule, o.brick_waves) == best[:3] + best[4:]
    assert np.array_equal(B.params.download(), before) and B.params.step == 0
    assert g.autotune(ctx, cat, batch=B, reps=2) == []          # cached
    # the tuned configuration computes the same thing
    out = g.batch_evaluate(ctx, B).cpu().numpy()
    grid = VOLUMES[0][0]
    V, A, bracket = F.evaluate_windowed(thetas[0], grid, 3.0, band=BAND)
    check_field(out[:B.voxel_offsets[1]].reshape(grid.shape), V, A, bracket)
    # single-volume tuning
    p = g.Params(ctx, VOLUMES[2][1]).upload(thetas[2].astype(np.float32))
    t1 = g.autotune(ctx, torch.from_numpy(fields[2]).cuda(), params=p,
                    grid=_ggrid(g, VOLUMES[2][0]), reps=1)
    assert len(t1) == 30


def test_automatic_brick_shape():
    """options.brick = 0: 8x8x32 bricks in XCD chunks until a call with a
    target field tunes the workload; the tuned choice is then used by every
    call on that workload (evaluation included), and the loss and gradient
    are those of the oracle whatever shape was chosen."""
    g, torch = _lib()
    grid, n, seed = VOLUMES[2]
    theta = _params(grid, n, seed)
    field = _field(grid, seed)
    ctx = g.Context(k=3.0, brick=0, deterministic=True)
    p = g.Params(ctx, n).upload(theta.astype(np.float32))
    gg, ft = _ggrid(g, grid), torch.from_numpy(field).cuda()

    def choice():
        st = ctx.stats()
        return st["bin_brick"], st["bin_brick_z"], st["bin_schedule"]

    g.evaluate(ctx, p, gg)
    assert choice() == (8, 32, 1)
    grad = torch.empty((11, n), device="cuda")
    L = g.loss_grad(ctx, p, ft, gg, grad)
    tuned = choice()
    assert tuned[:2] in {(8, 8), (8, 16), (8, 32), (16, 16)} and tuned[2] in (0, 1, 2)
    assert ctx.options.brick == 0                                 # stays automatic
    Lr, gr = F.loss_grad(theta, field.astype(np.float64), grid, 3.0)
    assert abs(L - Lr) <= 1e-5 * Lr
    slack, _ = F.boundary_slack(theta, field, grid, 3.0, BAND)
    check_grad(grad.cpu().numpy().astype(np.float64), gr, slack=slack)
    # the kept choice: no second tuning, the same deterministic result
    grad2 = torch.empty((11, n), device="cuda")
    assert g.loss_grad(ctx, p, ft, gg, grad2) == L
    assert torch.equal(grad2, grad) and choice() == tuned
    g.evaluate(ctx, p, gg)
    assert choice() == tuned
    g.refine(ctx, p, ft, gg, 2)                                   # refinement too
    assert choice() == tuned


def test_bad_batch_arguments():
    g, torch = _lib()
    ctx = g.Context()
    with pytest.raises(g.GveError):
        g.Batch(ctx, [g.Grid(8, 8, 8)], [0])
    with pytest.raises(g.GveError):
        g.Batch(ctx, [g.Grid(8, 0, 8)], [5])
    with pytest.raises(g.GveError):
        g.Batch(ctx, [], [])


def test_schedules_bitwise_equal_when_xcd_chunks_remap():
    """The XCD chunk schedule remaps bricks only when there are at least
    8 x 256 of them: 8^3 bricks on 136 x 128 x 128 voxels give 17 x 16 x 16 =
    4,352 bricks, two whole rounds of chunks plus a 256-brick tail.  Field,
    loss, gradient and three refinement steps (deterministic sums) are
    bitwise equal under all three schedules, and the field matches the oracle."""
    g, torch = _lib()
    grid = F.Grid(136, 128, 128)
    n = 6000
    print(f"schedules on {grid} n={n} (4352 bricks of 8^3)", flush=True)
    theta = S.random_params(n, (136, 128, 128), seed=31, scale_range=(0.8, 3.0))
    theta = theta.astype(np.float32)
    field = np.random.default_rng(32).uniform(size=grid.shape).astype(np.float32)
    ft = torch.from_numpy(field).cuda()
    gg = _ggrid(g, grid)
    res = []
    for sched in (0, 1, 2):
        ctx = g.Context(k=3.0, lr=5e-3, brick=8, brick_z=8, schedule=sched, deterministic=True)
        p = g.Params(ctx, n).upload(theta)
        out = g.evaluate(ctx, p, gg).cpu().numpy()
        assert ctx.stats()["n_bricks"] == 4352
        grad = torch.empty((11, n), device="cuda")
        L = g.loss_grad(ctx, p, ft, gg, grad)
        h = g.refine(ctx, p, ft, gg, 3)
        res.append((out, L, grad.cpu().numpy(), h, p.download()))
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0])
        assert r[1] == res[0][1]
        assert np.array_equal(r[2], res[0][2])
        assert np.array_equal(r[3], res[0][3])
        assert np.array_equal(r[4], res[0][4])
    V, A, bracket = F.evaluate_windowed(theta.astype(np.float64), grid, 3.0, band=BAND)
    check_field(res[1][0], V, A, bracket)
