"""GPU parity of the warm-start network, its features and targets vs the oracle.

The device computes every GEMM with bfloat16 operands on the matrix cores and
float32 accumulation; the oracle rounds the same operands to bfloat16 and
accumulates in float64.  Activations that land near a bfloat16 rounding
boundary may round the other way on one side, so the comparison is
norm-wise: outputs within 1e-3, gradients within 1e-2 per tensor.
"""
import numpy as np
import pytest

from oracle import alloc as A
from oracle import field as F
from oracle import mlp as Mo
from synth import fields as S

pytestmark = pytest.mark.gpu


def _lib():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    return g, torch


def _flat(p, fmean=None, fstd=None, tmean=None, tstd=None):
    parts = [p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"],
             np.zeros(16) if fmean is None else fmean, np.ones(16) if fstd is None else fstd,
             np.zeros(11) if tmean is None else tmean, np.ones(11) if tstd is None else tstd]
    return np.concatenate(parts).astype(np.float32)


def _net(seed):
    p = Mo.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, size=p[k].shape)
    # the device holds float32 weights; give the oracle the same values
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


@pytest.mark.parametrize("n", [1, 37, 1000, 70000])
def test_forward_matches_bf16_oracle(n):
    g, torch = _lib()
    p = _net(3)
    X = np.random.default_rng(n).normal(size=(n, 16)).astype(np.float32)
    ctx = g.Context()
    m = g.MLP(ctx, seed=0)
    m.load(_flat(p))
    Y = g.mlp_forward(ctx, m, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    Yr, _ = Mo.forward(p, X.astype(np.float64), bf16=True)
    assert np.linalg.norm(Y - Yr) <= 1e-3 * np.linalg.norm(Yr)


@pytest.mark.parametrize("n", [50, 4096])
def test_loss_and_gradients_match_bf16_oracle(n):
    g, torch = _lib()
    p = _net(5)
    rng = np.random.default_rng(9)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    T = rng.normal(size=(n, 11)).astype(np.float32)
    ctx = g.Context()
    m = g.MLP(ctx, seed=0)
    m.load(_flat(p))
    L, grad = g.mlp_loss_grad(ctx, m, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    grad = grad.cpu().numpy().astype(np.float64)
    Lr, gr = Mo.loss_and_grads(p, X.astype(np.float64), T.astype(np.float64), bf16=True)
    assert abs(L - Lr) <= 1e-3 * Lr
    off = 0
    for name, shape in g.MLP_LAYOUT:
        size = int(np.prod(shape))
        a, b = grad[off:off + size], gr[name].ravel()
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), name
        off += size


def test_training_reduces_loss_and_is_reproducible():
    g, torch = _lib()
    rng = np.random.default_rng(0)
    n = 20000
    X = rng.normal(size=(n, 16)).astype(np.float32) * 3 + 1
    W = rng.normal(size=(16, 11))
    T = (np.tanh(X @ W / 4) + 0.05 * rng.normal(size=(n, 11))).astype(np.float32)
    ctx = g.Context()
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m1 = g.MLP(ctx, seed=4)
    h1 = g.mlp_train(ctx, m1, Xt, Tt, epochs=8, batch=1024, lr=2e-3, seed=7)
    m2 = g.MLP(ctx, seed=4)
    h2 = g.mlp_train(ctx, m2, Xt, Tt, epochs=8, batch=1024, lr=2e-3, seed=7)
    assert h1[-1] < 0.5 * h1[0]
    assert np.array_equal(h1, h2) and np.array_equal(m1.export(), m2.export())
    st = m1.tensors()
    assert np.allclose(st["fmean"], X.mean(axis=0), atol=1e-4)
    assert np.allclose(st["tstd"], T.std(axis=0), rtol=1e-4)


def test_features_and_targets_match_oracle():
    g, torch = _lib()
    f, _ = S.tiny_mixture(seed=0, normalize=True)
    grid = F.Grid(64, 64, 64)
    ctx = g.Context(k=3.0)
    ft = torch.from_numpy(f).cuda()
    P, info = g.allocate(ctx, ft, g.Grid(64, 64, 64), 2048, 11)
    theta = P.download().astype(np.float64)
    X = g.features(ctx, P, ft, g.Grid(64, 64, 64), info["n_detail"], info["g99"]).cpu().numpy()
    Xr = Mo.features(f, grid, theta, info["n_detail"], info["g99"], 3.0)
    # eigenvalue features, gradient ratio, box mean/variance, group flag
    assert np.max(np.abs(X[:, 0:3] - Xr[:, 0:3])) < 1e-4
    assert np.max(np.abs(X[:, 12] - Xr[:, 12])) < 1e-5 * max(1.0, np.max(np.abs(Xr[:, 12])))
    assert np.max(np.abs(X[:, 13] - Xr[:, 13])) < 1e-5
    assert np.max(np.abs(X[:, 14] - Xr[:, 14])) < 1e-5
    assert np.array_equal(X[:, 15], Xr[:, 15])
    # eigenvectors where the eigenvalues are separated
    lam = np.expm1(Xr[:, 0:3])
    ok = (lam[:, 0] - lam[:, 1] > 1e-3 * lam[:, 0]) & (lam[:, 1] - lam[:, 2] > 1e-3 * lam[:, 0])
    assert ok.mean() > 0.5
    assert np.max(np.abs(X[ok, 3:12] - Xr[ok, 3:12])) < 1e-4
    # targets of a perturbed copy
    ref = theta.copy()
    ref[0:3] += 0.25
    ref[3:7] *= -1.5
    ref[10] *= 1.1
    Q = g.Params(ctx, 2048).upload(ref.astype(np.float32))
    T = g.targets(ctx, P, Q).cpu().numpy()
    Tr = Mo.targets(theta, ref.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(T - Tr)) < 1e-6


def test_warmstart_never_worse_than_allocation():
    g, torch = _lib()
    f, _ = S.tiny_mixture(seed=1, normalize=True)
    ctx = g.Context(k=3.0, lr=1e-3)
    ft = torch.from_numpy(f).cuda()
    grid = g.Grid(64, 64, 64)
    P, info = g.allocate(ctx, ft, grid, 2048, 5)
    before = P.download()
    L0 = g.loss_grad(ctx, P, ft, grid)
    m = g.MLP(ctx, seed=3)          # untrained: its correction is noise
    applied, L = g.warmstart(ctx, m, P, ft, grid, info["n_detail"], info["g99"])
    after_loss = g.loss_grad(ctx, P, ft, grid)
    assert abs(L[0] - L0) <= 1e-9 * L0
    assert after_loss <= L0 * (1 + 1e-9)
    if applied == 0:
        assert np.array_equal(P.download(), before)
    else:
        assert abs(after_loss - L[applied]) <= 1e-9 * L0
    assert P.step == 0
