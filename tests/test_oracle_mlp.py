"""Pins for the warm-start oracle (CPU only): bfloat16 rounding, GELU, the
network's gradients, Adam, features and targets."""
import math

import numpy as np
import pytest

from oracle import alloc as A
from oracle import field as F
from oracle import mlp as Mo


def test_bf16_round_ties_to_even_and_matches_torch():
    assert Mo.bf16_round(np.array([1.0]))[0] == 1.0
    assert Mo.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0           # tie -> even
    assert Mo.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.015625  # tie -> even (up)
    assert Mo.bf16_round(np.array([1.0 + 2 ** -8 + 2 ** -12]))[0] == 1.0078125
    assert Mo.bf16_round(np.array([-3.0]))[0] == -3.0
    import torch

    x = np.random.default_rng(0).normal(0, 10, size=10000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(Mo.bf16_round(x), ref)


def test_gelu_values_and_derivative():
    assert Mo.gelu(np.array([0.0]))[0] == 0.0
    assert abs(Mo.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # Phi(1)
    assert abs(Mo.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15
    assert abs(Mo.gelu(np.array([12.0]))[0] - 12.0) < 1e-12
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (Mo.gelu(z + h) - Mo.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - Mo.gelu_grad(z))) < 1e-9


def test_network_gradients_match_central_differences():
    p = Mo.init_params(3)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(7, Mo.D_IN))
    T = rng.normal(size=(7, Mo.D_OUT))
    L, g = Mo.loss_and_grads(p, X, T)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].ravel()
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for j in idx:
            h = 1e-6
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name].ravel()[j] += h
            pm[name].ravel()[j] -= h
            fd = (Mo.loss_and_grads(pp, X, T)[0] - Mo.loss_and_grads(pm, X, T)[0]) / (2 * h)
            assert abs(fd - g[name].ravel()[j]) < 1e-7 * max(1.0, abs(fd)), (name, j)


def test_he_uniform_bounds_and_bf16_forward_close_to_exact():
    p = Mo.init_params(5)
    assert np.max(np.abs(p["W1"])) <= math.sqrt(6 / 16)
    assert np.max(np.abs(p["W2"])) <= math.sqrt(6 / 128)
    X = np.random.default_rng(2).normal(size=(64, 16))
    Y, _ = Mo.forward(p, X)
    Yb, _ = Mo.forward(p, X, bf16=True)
    rel = np.linalg.norm(Yb - Y) / np.linalg.norm(Y)
    assert 1e-5 < rel < 2e-2      # bf16 operands: ~3 significant digits


def test_adam_step_one():
    p = {"W": np.array([[0.5, -0.2]])}
    g = {"W": np.array([[0.3, -0.7]])}
    out = Mo.adam(p, g, {}, lr=1e-3)
    assert np.allclose(out["W"], p["W"] - 1e-3 * np.sign(g["W"]), atol=1e-10)


def test_features_of_a_planar_front_and_constant_box():
    n = 24
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    f = (0.5 * (1 + np.tanh((x - 11.6) / 2.5))).astype(np.float32)
    grid = F.Grid(n, n, n)
    p = np.zeros((11, 2))
    p[0:3, 0] = (12.2, 11.9, 12.1)
    p[0:3, 1] = (3.0, 12.0, 12.0)
    p[3] = 1.0
    p[7:10] = np.log(1.5)
    X = Mo.features(f, grid, p, n_detail=1, g99=0.1, k=3.0)
    assert abs(abs(X[0, 3]) - 1.0) < 1e-6                  # e1 = +x (front normal)
    assert X[0, 3] > 0 and X[0, 15] == 1.0 and X[1, 15] == 0.0
    assert X[0, 0] > X[0, 1] >= X[0, 2] >= 0.0             # log1p(eigenvalues)
    g32 = A.gradient_magnitude32(f)
    assert abs(X[0, 12] - g32[12, 12, 12] / 0.1) < 1e-6
    c = np.full((10, 10, 10), 0.37, dtype=np.float32)
    Xc = Mo.box_stats(c, F.Grid(10, 10, 10), p[:, :1] * 0 + np.array([[5], [5], [5], [1], [0], [0], [0], [0.0], [0.0], [0.0], [1]]), 3.0)
    assert abs(Xc[0, 0] - 0.37) < 1e-7 and abs(Xc[0, 1]) < 1e-12


def test_targets_align_quaternion_sign():
    a = np.zeros((11, 2))
    a[3] = (1.0, 0.6)
    a[4] = (0.0, 0.8)
    r = a.copy()
    r[3:7, 0] *= -2.0                  # same rotation, opposite sign, not unit
    r[0, 1] += 0.5
    T = Mo.targets(a, r)
    assert np.allclose(T[0], 0.0, atol=1e-15)
    assert abs(T[1, 0] - 0.5) < 1e-15 and np.allclose(T[1, 1:], 0.0, atol=1e-15)
