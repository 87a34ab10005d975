"""Pins for the allocation oracle (CPU only).

Fixed against: the published SplitMix64 test vector, the paper's seed-limit
arithmetic (Sec. V-B: 125,787 eligible voxels support about 2.3e5 primitives at
55 % detail), sampling statistics of the two draws, closed-form gradients and
structure tensors of analytic fields, lattice spacings, and least squares.
"""
import math

import numpy as np
import pytest

from oracle import alloc as A
from oracle import field as F
from synth import fields as S


def test_splitmix64_reference_vector():
    # First two outputs of the SplitMix64 generator started from state 0.
    assert int(A.splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    assert int(A.splitmix64(np.uint64(0x9E3779B97F4A7C15))) == 0x6E789E6AA1B965F4


def test_uniform_is_in_unit_interval_and_counter_based():
    u = A.uniform01(7, 3, np.arange(100000))
    assert u.min() > 0 and u.max() <= 1
    assert abs(u.mean() - 0.5) < 0.005
    assert np.array_equal(u[1234:1240], A.uniform01(7, 3, np.arange(1234, 1240)))
    assert not np.array_equal(u[:10], A.uniform01(7, 4, np.arange(10)))


def test_budget_split_and_seed_limit_arithmetic():
    assert A.split_budget(2048) == (1126, 922)
    assert A.split_budget(1_400_000) == (770_000, 630_000)
    # Sec. V-B: 125,787 eligible voxels -> about 2.3e5 primitives (0.55 N <= 125,787)
    nmax = A.max_feasible_budget(125_787, 10 ** 9)
    assert nmax == 228_704
    assert round(nmax, -4) == 230_000
    d, c = A.split_budget(nmax + 1)
    assert d == 125_788


def test_infeasible_budget_reports_shortfall():
    f = np.zeros((8, 8, 8), np.float32)
    f[2:4, 2:4, 2:4] = 1.0                   # 8 occupied voxels
    g32 = A.gradient_magnitude32(f)
    with pytest.raises(A.BudgetInfeasible) as e:
        A.draw_seeds(f, g32, 40, seed=1)
    n_det, n_cov = A.split_budget(40)
    assert e.value.n_occupied == 8
    assert e.value.shortfall == max(n_det - e.value.n_eligible, n_cov - 8)


def test_gradient_matches_analytic_ramp_and_p99():
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(9), indexing="ij")
    f = (0.03 * x + 0.02 * y - 0.01 * z + 0.3).astype(np.float32)
    g = A.gradient_magnitude32(f)
    exact = math.sqrt(0.03 ** 2 + 0.02 ** 2 + 0.01 ** 2)
    assert np.max(np.abs(g - exact)) < 2e-7
    assert abs(A.percentile_order_stat(g) - exact) < 2e-7


def test_detail_draw_is_proportional_to_gradient():
    # piecewise-linear in x: slope 0.001 on the left half, 0.003 on the right
    n = 64
    x = np.arange(n, dtype=np.float64)
    prof = np.where(x < n // 2, 0.5 + 0.001 * x, 0.5 + 0.001 * (n // 2) + 0.003 * (x - n // 2))
    f = np.broadcast_to(prof.astype(np.float32), (n, n, n)).copy()
    g32 = A.gradient_magnitude32(f)
    det, cov, _, _ = A.draw_seeds(f, g32, 4000, seed=3)
    right = (det % n) >= n // 2
    # small sample (2,200 of 262,144): inclusion probability ~ proportional to g
    gw = g32.astype(np.float64).reshape(n, n, n)
    p = gw[:, :, n // 2:].sum() / gw.sum()
    assert abs(p - 0.75) < 0.02
    assert abs(right.mean() - p) < 4 * math.sqrt(p * (1 - p) / det.size)
    frac_cov = np.mean((cov % n) >= n // 2)
    assert abs(frac_cov - 0.5) < 4 * math.sqrt(0.25 / cov.size)
    assert np.unique(det).size == det.size and np.unique(cov).size == cov.size


def test_draws_respect_domains_and_jitter_bounds():
    f, _ = S.tiny_mixture(seed=2, n=32, count=40, normalize=True)
    g32 = A.gradient_magnitude32(f)
    det, cov, ne, no = A.draw_seeds(f, g32, 600, seed=5)
    v = f.ravel()
    assert np.all(v[det] > 0.02) and np.all(g32.ravel()[det] > 0)
    assert np.all(v[cov] > 0.02)
    mu = A.jitter_centers(det, f.shape, (0, 0, 0), 5, 0)
    i, j, k = det % 32, (det // 32) % 32, det // 1024
    for a, base in enumerate((i, j, k)):
        off = mu[a].astype(np.float64) - base
        assert np.all(off >= -0.5) and np.all(off <= 0.5)


def test_spacing_of_a_lattice():
    h = 2.5
    pts = np.stack(np.meshgrid(np.arange(6), np.arange(7), np.arange(5), indexing="ij")).reshape(3, -1)
    mu = (pts * h + 0.25).astype(np.float32)
    assert abs(A.group_spacing(mu) - h) < 1e-6


def test_structure_tensor_of_planar_front():
    n = 24
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    nrm = np.array([0.48, -0.6, 0.64])
    nrm /= np.linalg.norm(nrm)
    s = (x - 11.3) * nrm[0] + (y - 12.1) * nrm[1] + (z - 11.7) * nrm[2]
    f = (0.5 * (1 + np.tanh(s / 3.0))).astype(np.float32)
    parts = A.gradient_parts(f)
    J = A.structure_tensor(parts, (12, 12, 12))
    R, lam = A.frame_from_tensor(J)
    assert abs(abs(R[:, 2] @ nrm) - 1) < 2e-3          # e1 (largest) = front normal
    assert abs(R[:, 0] @ nrm) < 5e-2                     # tangent lies in the front
    assert lam[0] > 50 * lam[1]
    assert np.allclose(R.T @ R, np.eye(3), atol=1e-12) and np.linalg.det(R) > 0


def test_quaternion_round_trip():
    rng = np.random.default_rng(0)
    for _ in range(50):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = F.rotation(q)
        q2 = A.quat_from_rotation(R)
        assert np.allclose(F.rotation(q2), R, atol=1e-12)
        assert q2[0] >= 0


def test_lsq_weight():
    rng = np.random.default_rng(1)
    U = rng.uniform(size=1000)
    assert abs(A.lsq_weight(U, 2.5 * U) - 2.5) < 1e-12
    V = 2.5 * U + rng.normal(0, 0.1, size=1000)
    k = A.lsq_weight(U, V)
    assert abs(k - np.polyfit(U, V, 1, full=False)[0]) < 0.5   # sanity vs slope fit
    assert abs(((U * k - V) * U).sum()) < 1e-9                 # normal equation


def test_allocate_tiny_workload_invariants():
    f, _ = S.tiny_mixture(seed=0, normalize=True)
    grid = F.Grid(64, 64, 64)
    params, info = A.allocate(f, grid, 2048, seed=11, k=3.0)
    assert params.shape == (11, 2048)
    assert (info.n_det, info.n_cov) == (1126, 922)
    # scales: detail tighter than coverage; elongation within [1, 3]; cap 64/16 = 4
    assert info.s_base[0] < info.s_base[1]
    s = np.exp(params[7:10])
    assert np.all(s >= 0.25 - 1e-12) and np.all(s <= 4.0 + 1e-12)
    ratio = s[0] / s[1]
    assert np.all(ratio >= 1 - 1e-12) and np.all(ratio <= 3 + 1e-12)
    qn = np.linalg.norm(params[3:7], axis=0)
    assert np.allclose(qn, 1.0, atol=1e-12)
    # the least-squares weight makes the allocated field a better fit than zero
    V, _ = F.evaluate_windowed(params, grid, 3.0)
    assert np.sum((V - f) ** 2) < np.sum(f.astype(np.float64) ** 2)
    assert info.kappa > 0
