"""GPU parity of the learned warm start's application and of the network's
training step against the oracle (``oracle.mlp.warmstart``, ``oracle.mlp.train``).

Warm start: the library applies theta += alpha Delta for alpha = 1, 1/2, 1/4
and keeps the first alpha whose full-grid loss is below the unchanged set's
(else it falls back to the allocation).  The inputs are a planted problem: the
target is the truncated field of a random primitive set theta* plus noise, and
the set handed to the warm start is theta* with every log-scale lowered by 0.1,
so a correction of +0.1 s on the log-scales overshoots by a known factor s.
A network whose last layer is zero outputs its bias exactly, so Delta is known
exactly on both sides and every branch of the retry logic is reached: s = 1
(alpha 1 kept), 2.5 (alpha 1/2), 5 (alpha 1/4) and 10 (fallback).  A network
with a random last layer checks the per-primitive mapping of the outputs
through the features.  Losses within 1e-5 relative; parameters to float32
rounding (or the network's bfloat16 tolerance).

Training: one full-batch epoch, three full-batch epochs and two mini-batch
epochs from the device's own initial weights, compared with the bfloat16-
emulating oracle (standardisation, epoch permutation, Adam).
"""
import math

import numpy as np
import pytest

from oracle import field as F
from oracle import mlp as Mo
from synth import fields as S
from tests.parity import BAND

pytestmark = pytest.mark.gpu

K = 3.0
N = 2048
GRID = F.Grid(64, 64, 64)


def _lib():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    return g, torch


def _planted():
    star = S.random_params(N, 64, seed=21, scale_range=(1.5, 4.0)).astype(np.float32)
    star = star.astype(np.float64)
    V, _ = F.evaluate_windowed(star, GRID, K)
    V = V + np.random.default_rng(22).normal(0.0, 0.01, size=V.shape)
    V = V.astype(np.float32)
    theta = star.copy()
    theta[7:10] -= 0.1
    theta = theta.astype(np.float32).astype(np.float64)
    return V, theta


def _loss_fn(V):
    # the device stores parameters in float32: both sides decide on float32 sets
    return lambda th: F.loss(np.asarray(th).astype(np.float32).astype(np.float64), V, GRID, K)


def _flat(p, fmean, fstd, tmean, tstd):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"],
                           p["W3"].ravel(), p["b3"], fmean, fstd, tmean, tstd]).astype(np.float32)


def _constant_net(delta, seed):
    """A network whose output is its last bias: W3 = 0.  Returns (params, flat,
    tmean, tstd) with tmean + b3 * tstd = delta."""
    rng = np.random.default_rng(seed)
    p = Mo.init_params(seed)
    p["W3"][:] = 0.0
    p["b3"] = rng.normal(size=11)
    tstd = rng.uniform(0.5, 2.0, size=11)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    tstd = tstd.astype(np.float32).astype(np.float64)
    tmean = (delta - p["b3"] * tstd).astype(np.float32).astype(np.float64)
    return p, _flat(p, np.zeros(16), np.ones(16), tmean, tstd), tmean, tstd


def _run_gpu(g, torch, V, theta, flat, n_detail, g99):
    ctx = g.Context(k=K)
    P = g.Params(ctx, N).upload(theta.astype(np.float32))
    m = g.MLP(ctx, seed=0)
    m.load(flat)
    ft = torch.from_numpy(V).cuda()
    applied, L = g.warmstart(ctx, m, P, ft, g.Grid(64, 64, 64), n_detail, g99)
    return applied, L, P.download().astype(np.float64), P.step


@pytest.mark.parametrize("scale,expect", [(1.0, 1), (2.5, 2), (5.0, 3), (10.0, 0)])
def test_warmstart_matches_oracle_on_every_branch(scale, expect):
    g, torch = _lib()
    print(f"warmstart planted 64^3 x {N}, overshoot {scale}", flush=True)
    V, theta = _planted()
    delta = np.zeros(11)
    delta[7:10] = 0.1 * scale
    p, flat, tmean, tstd = _constant_net(delta, seed=int(10 * scale))
    Y = np.tile(p["b3"], (N, 1))
    applied_r, L_r, th_r = Mo.warmstart(theta, Y, tmean, tstd, _loss_fn(V))
    # the designed branch is reached, with decisions far from the tolerance
    assert applied_r == expect, (applied_r, L_r)
    tried = applied_r if applied_r else 3
    for j in range(1, tried + 1):
        assert abs(L_r[j] - L_r[0]) > 1e-3 * L_r[0]
    applied, L, th, step = _run_gpu(g, torch, V, theta, flat, n_detail=N // 2, g99=0.05)
    assert applied == applied_r
    for j in range(4):
        if math.isnan(L_r[j]):
            assert math.isnan(L[j])
        else:
            assert abs(L[j] - L_r[j]) <= 1e-5 * L_r[j], (j, L[j], L_r[j])
    # theta: float32 rounding of base + alpha * (b3 tstd + tmean)
    assert np.max(np.abs(th - th_r) / (np.abs(th_r) + 1e-6)) < 4e-7
    if applied == 0:
        assert np.array_equal(th, theta.astype(np.float32).astype(np.float64))
    assert step == 0


def test_warmstart_random_network_maps_outputs_per_primitive():
    """Random hidden layers and last layer: Delta varies per primitive through
    the features; its mean lifts the log-scales by 0.1 (accepted at alpha 1).
    The eigenvector features are given zero weight (where eigenvalues are
    nearly equal their sign/rotation is not unique)."""
    g, torch = _lib()
    print(f"warmstart random network 64^3 x {N}", flush=True)
    V, theta = _planted()
    rng = np.random.default_rng(5)
    p = Mo.init_params(7)
    p["W1"][:, 3:12] = 0.0
    p["b1"] = rng.normal(0, 0.1, size=128)
    p["b2"] = rng.normal(0, 0.1, size=128)
    p["W3"] *= 0.5
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    n_detail, g99 = 1000, 0.05
    X = Mo.features(V, GRID, theta, n_detail, g99, K)
    fmean, fstd = Mo.column_stats(X)
    fmean = fmean.astype(np.float32).astype(np.float64)
    fstd = fstd.astype(np.float32).astype(np.float64)
    tstd = np.full(11, 2e-3)
    tmean = np.zeros(11)
    tmean[7:10] = 0.1
    Yr, _ = Mo.forward(p, (X - fmean) / fstd, bf16=True)
    applied_r, L_r, th_r = Mo.warmstart(theta, Yr, tmean, tstd, _loss_fn(V))
    assert applied_r == 1 and L_r[0] - L_r[1] > 1e-2 * L_r[0]
    applied, L, th, _ = _run_gpu(g, torch, V, theta, _flat(p, fmean, fstd, tmean, tstd),
                                 n_detail, g99)
    assert applied == 1
    assert abs(L[0] - L_r[0]) <= 1e-5 * L_r[0]
    assert abs(L[1] - L_r[1]) <= 1e-4 * L_r[1]
    # the per-primitive part of the correction (mean removed) agrees to the
    # network's bfloat16 tolerance, entry by entry for most primitives
    d = th - theta - tmean[:, None]
    dr = th_r - theta - tmean[:, None]
    assert np.linalg.norm(d - dr) <= 2e-2 * np.linalg.norm(dr)
    assert np.linalg.norm(dr) > 0.1 * np.linalg.norm(2e-3 * Yr)


def _train_data(n, seed):
    rng = np.random.default_rng(seed)
    X = (rng.normal(size=(n, 16)) * 3.0 + 1.0).astype(np.float32)
    W = rng.normal(size=(16, 11))
    T = (np.tanh(X @ W / 4.0) + 0.05 * rng.normal(size=(n, 11))).astype(np.float32)
    return X, T


def _grad_clear(p, X, T, stats):
    """Entries whose first-step gradient is far from zero (their Adam step
    cannot change sign between two correct roundings)."""
    fm, fs, tm, ts = stats
    _, gr = Mo.loss_and_grads(p, (X - fm) / fs, (T - tm) / ts, bf16=True)
    return {k: np.abs(v) > 1e-2 * np.max(np.abs(v)) for k, v in gr.items()}


@pytest.mark.parametrize("epochs,batch", [(1, 3000), (3, 3000), (2, 1024)])
def test_training_matches_oracle(epochs, batch):
    g, torch = _lib()
    n, lr, seed = 3000, 1e-3, 17
    print(f"mlp_train n={n} epochs={epochs} batch={batch}", flush=True)
    X, T = _train_data(n, 4)
    ctx = g.Context()
    m = g.MLP(ctx, seed=9)
    w0 = m.export().astype(np.float64)
    p0 = Mo.flat_to_params(w0)
    hist = g.mlp_train(ctx, m, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(),
                       epochs=epochs, batch=batch, lr=lr, seed=seed)
    got = m.tensors()
    pr, stats, hist_r = Mo.train(p0, X.astype(np.float64), T.astype(np.float64), epochs, batch,
                                 lr, seed, bf16=True)
    fm, fs, tm, ts = stats
    assert np.allclose(got["fmean"], fm, rtol=1e-6, atol=1e-7)
    assert np.allclose(got["fstd"], fs, rtol=1e-6)
    assert np.allclose(got["tmean"], tm, rtol=1e-6, atol=1e-7)
    assert np.allclose(got["tstd"], ts, rtol=1e-6)
    assert np.allclose(hist, hist_r, rtol=1e-3)
    clear = _grad_clear(p0, X.astype(np.float64), T.astype(np.float64), stats)
    wn = dn = en = 0.0
    for k in p0:
        dw, dwr = got[k] - p0[k], pr[k] - p0[k]
        wn += float(np.sum(pr[k] ** 2))
        dn += float(np.sum(dwr ** 2))
        en += float(np.sum((dw - dwr) ** 2))
        if epochs == 1:
            # one Adam step: lr g / (|g| + eps) entry by entry where g is clear
            assert np.max(np.abs(dw - dwr)[clear[k]]) <= 1e-3 * lr, k
    print(f"weights rel {math.sqrt(en / wn):.2e}, update rel {math.sqrt(en / dn):.2e}")
    assert math.sqrt(en / wn) <= 1e-3
    assert math.sqrt(en / dn) <= 5e-2


def test_count_pairs_matches_oracle():
    """In-support (primitive, voxel) pairs counted on the device equal the
    oracle's count up to the pairs whose float64 m^2 lies within the band of
    the cut (those float32 may decide either way)."""
    g, torch = _lib()
    cases = [(F.Grid(37, 29, 21, 3, -2, 5), 60, 0, (0.6, 4.0)),
             (F.Grid(64, 64, 64), N, 7, (1.5, 4.0))]
    for grid, n, seed, sr in cases:
        print(f"count_pairs grid={grid} n={n}", flush=True)
        p = S.random_params(n, (grid.nx, grid.ny, grid.nz), seed=seed, scale_range=sr,
                            unit_quat=False)
        p[0] += grid.x0 + np.random.default_rng(seed).uniform(-3, 3, n)
        p[1] += grid.y0
        p[2] += grid.z0
        p = p.astype(np.float32).astype(np.float64)
        ref = F.count_pairs(p, grid, K)
        _, _, (_, _, namb) = F.evaluate_windowed(p, grid, K, band=BAND)
        for shape in ((8, 32), (8, 8), (16, 16)):
            ctx = g.Context(k=K, brick=shape[0], brick_z=shape[1])
            P = g.Params(ctx, n).upload(p.astype(np.float32))
            nin, ncand = g.count_pairs(ctx, P, g.Grid(grid.nx, grid.ny, grid.nz, grid.x0,
                                                       grid.y0, grid.z0))
            assert abs(nin - ref) <= namb, (shape, nin, ref, namb)
            assert ncand >= nin
