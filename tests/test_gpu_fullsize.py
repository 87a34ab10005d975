"""Parity at the benchmark's full size: 1024^3 fronts field, 1.4M primitives
from the device allocation, k = 3, the benchmark's launch configuration
(default options: 8x8x32 bricks, XCD chunk schedule, atomic sums).

The oracle cannot evaluate a billion voxels, so it checks samples it can
compute one by one: the field at sampled voxels (from every primitive whose
support box holds the voxel), and the loss gradient of sampled primitives (on
a sub-grid covering each one's support box, with every primitive whose box
meets that sub-grid, which is exactly the data its gradient depends on).

Besides uniform samples, both tests take the cases a brick kernel is most
likely to get wrong: voxels on the grid's corners and faces and on brick
edges (x, y at 0 or 7 modulo 8, z at 0 or 31 modulo 32), primitives whose
support box the grid clips, and the largest and smallest support boxes.
"""
import math

import numpy as np
import pytest

from oracle import field as F
from synth import fields as S
from tests.parity import BAND, check_field, check_grad

pytestmark = pytest.mark.gpu

N_SIDE = 1024
BUDGET = 1_400_000
SEED = 2026


@pytest.fixture(scope="module")
def workload():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    print("[fullsize] fronts 1024^3 + allocation of 1.4M", flush=True)
    field = S.fronts_field(N_SIDE, SEED, device="cuda")
    grid = g.Grid(N_SIDE, N_SIDE, N_SIDE)
    ctx = g.Context(k=3.0)
    P, info = g.allocate(ctx, field, grid, BUDGET, SEED)
    theta = P.download().astype(np.float64)
    return g, torch, ctx, field, grid, P, theta


def _boxes(theta, k):
    """Support boxes (inclusive voxel ranges, unclipped) of every primitive."""
    S_ = F.covariance(theta)
    half = k * np.sqrt(np.stack([S_[:, 0, 0], S_[:, 1, 1], S_[:, 2, 2]], axis=1))
    mu = theta[0:3].T
    return np.ceil(mu - half).astype(np.int64), np.floor(mu + half).astype(np.int64)


def _meets(lo, hi, a, b):
    """Primitives whose box meets the voxel box [a, b] (inclusive, per axis)."""
    return np.nonzero(np.all(lo <= b, axis=1) & np.all(hi >= a, axis=1))[0]


def _sample_voxels(rng):
    """Uniform voxels, the eight corners, voxels on each face and voxels on
    brick edges (8 x 8 x 32 bricks)."""
    e = N_SIDE - 1
    uniform = rng.integers(0, N_SIDE, size=(400, 3))
    corners = np.array([[x, y, z] for x in (0, e) for y in (0, e) for z in (0, e)])
    faces = rng.integers(0, N_SIDE, size=(60, 3))
    faces[np.arange(60), np.arange(60) % 3] = np.where(np.arange(60) % 2 == 0, 0, e)
    edges = 8 * rng.integers(0, N_SIDE // 8, size=(60, 3))
    edges[:, 0] += rng.choice([0, 7], size=60)
    edges[:, 1] += rng.choice([0, 7], size=60)
    edges[:, 2] = 32 * rng.integers(0, N_SIDE // 32, size=60) + rng.choice([0, 31], size=60)
    return np.concatenate([uniform, corners, faces, edges])


def _sample_primitives(rng, lo, hi):
    """Uniform primitives, primitives whose support box the grid clips, and
    the largest and smallest clipped boxes (largest among those of at most
    250,000 voxels, which the oracle visits in seconds)."""
    a = np.maximum(lo, 0)
    b = np.minimum(hi, N_SIDE - 1)
    vol = np.prod(np.maximum(b - a + 1, 0), axis=1)
    clipped = np.nonzero((np.any(lo < 0, axis=1) | np.any(hi > N_SIDE - 1, axis=1))
                         & (vol > 0))[0]
    picks = list(rng.choice(BUDGET, size=24, replace=False))
    if clipped.size:
        picks += list(rng.choice(clipped, size=min(6, clipped.size), replace=False))
    key = np.where(vol <= 250_000, vol, -1)
    order = np.argsort(key, kind="stable")
    picks += list(order[-3:]) + list(order[np.searchsorted(key[order], 1):][:3])
    print(f"[fullsize] {clipped.size} clipped boxes; picked boxes of {vol[order[-1]]} "
          f"and {vol[order[np.searchsorted(key[order], 1)]]} voxels", flush=True)
    return np.unique(np.array(picks, dtype=np.int64))


def test_field_at_sampled_voxels(workload):
    g, torch, ctx, field, grid, P, theta = workload
    out = g.evaluate(ctx, P, grid)
    lo, hi = _boxes(theta, 3.0)
    rng = np.random.default_rng(11)
    vox = _sample_voxels(rng)
    print(f"[fullsize] field at {len(vox)} voxels", flush=True)
    flat = out.reshape(-1)
    for x, y, z in vox:
        cand = _meets(lo, hi, np.array([x, y, z]), np.array([x, y, z]))
        sub = theta[:, cand]
        g1 = F.Grid(1, 1, 1, int(x), int(y), int(z))
        V, A, bracket = F.evaluate_windowed(sub, g1, 3.0, band=BAND)
        got = float(flat[int(x) + N_SIDE * (int(y) + N_SIDE * int(z))])
        check_field(np.array([[[got]]]), V, A, bracket)


def test_gradient_of_sampled_primitives(workload):
    g, torch, ctx, field, grid, P, theta = workload
    grad = torch.empty((11, BUDGET), device="cuda")
    g.loss_grad(ctx, P, field, grid, grad)
    grad = grad.cpu().numpy().astype(np.float64)
    lo, hi = _boxes(theta, 3.0)
    rng = np.random.default_rng(12)
    picks = _sample_primitives(rng, lo, hi)
    fld = field  # torch, on the device
    for i in picks:
        a = np.maximum(lo[i], 0)
        b = np.minimum(hi[i], N_SIDE - 1)
        sub_grid = F.Grid(int(b[0] - a[0] + 1), int(b[1] - a[1] + 1), int(b[2] - a[2] + 1),
                          int(a[0]), int(a[1]), int(a[2]))
        cand = _meets(lo, hi, a, b)
        j = int(np.nonzero(cand == i)[0][0])
        block = fld[a[2]:b[2] + 1, a[1]:b[1] + 1, a[0]:b[0] + 1].cpu().numpy().astype(np.float64)
        # coordinates relative to the sub-grid are the same world coordinates
        _, gr = F.loss_grad(theta[:, cand], block, sub_grid, 3.0)
        slack, _ = F.boundary_slack(theta[:, cand], block, sub_grid, 3.0, BAND)
        # one primitive's gradient sums thousands of float32 terms with heavy
        # cancellation (q . dL/dq = 0): its error scale is the absolute sum
        absg = F.loss_grad_absolute(theta[:, cand], block, sub_grid, 3.0)[:, j:j + 1]
        print(f"[fullsize] primitive {i}: {cand.size} neighbours, box {sub_grid.shape}", flush=True)
        rel = check_grad(grad[:, i:i + 1], gr[:, j:j + 1], slack=slack[:, j:j + 1], absolute=absg)
        ga = grad[:, i].astype(np.float64)
        ea = np.abs(ga - gr[:, j])
        print(f"[fullsize] primitive {i}: err/|g| per group "
              + ", ".join(f"{k} {v:.1e}" for k, v in rel.items())
              + f"; max entry err/|g| {np.max(ea / np.maximum(np.abs(gr[:, j]), 1e-30)):.1e}, "
              f"max entry err/A_g {np.max(ea / np.maximum(absg[:, 0], 1e-30)):.1e}", flush=True)


def test_refinement_with_asynchronous_binning_at_full_size(workload):
    """Deterministic sums at the benchmark's size: one refinement call of four
    iterations (binning sized on the device after the first) ends bitwise where
    four one-iteration calls (each binning sized on the host) end, losses
    included."""
    g, torch, _, field, grid, P, theta = workload
    print("[fullsize] refinement, asynchronous vs synchronous binning", flush=True)
    ctx = g.Context(k=3.0, deterministic=True)
    a = g.Params(ctx, BUDGET).upload(theta.astype(np.float32))
    la = g.refine(ctx, a, field, grid, 4)
    assert ctx.stats()["n_resized"] == 0
    ta = a.download()
    a.close()
    b = g.Params(ctx, BUDGET).upload(theta.astype(np.float32))
    lb = np.concatenate([g.refine(ctx, b, field, grid, 1) for _ in range(4)])
    tb = b.download()
    b.close()
    print(f"[fullsize] losses {la.tolist()}", flush=True)
    assert np.array_equal(la, lb)
    assert np.array_equal(ta, tb)
    assert la[-1] < la[0]
