"""Pins for the oracle's field, loss, gradient and Adam (CPU only).

Each test fixes the oracle against something other than itself: closed forms
of Gaussian integrals and lattice sums, the generator's independently written
Gaussian formula, symmetries of the quaternion parameterisation, central finite
differences, and the Adam update written out by hand.
"""
import math

import numpy as np
import pytest

from oracle import field as F
from synth import fields as S


def one(mu, q, s, c):
    p = np.zeros((11, 1))
    p[0:3, 0] = mu
    p[3:7, 0] = q
    p[7:10, 0] = np.log(np.asarray(s, dtype=np.float64))
    p[10, 0] = c
    return p


def q3_tail(k):
    """Mass of a standard 3-D Gaussian outside radius k (chi-3 survival)."""
    return math.erfc(k / math.sqrt(2.0)) + math.sqrt(2.0 / math.pi) * k * math.exp(-k * k / 2.0)


# --------------------------------------------------------------------------- values

def test_single_isotropic_closed_form():
    g = F.Grid(9, 10, 11)
    mu = (4.3, 5.1, 4.7)
    p = one(mu, (1, 0, 0, 0), (1.7, 1.7, 1.7), 0.8)
    zz, yy, xx = np.meshgrid(np.arange(11), np.arange(10), np.arange(9), indexing="ij")
    r2 = (xx - mu[0]) ** 2 + (yy - mu[1]) ** 2 + (zz - mu[2]) ** 2
    ref = 0.8 * np.exp(-r2 / (2 * 1.7 ** 2))
    assert np.max(np.abs(F.evaluate_bruteforce(p, g) - ref)) < 1e-15
    # truncated at k: the closed form with the strict cut applied
    for k in (2.0, 3.0):
        refk = np.where(r2 / 1.7 ** 2 < k * k, ref, 0.0)
        assert np.max(np.abs(F.evaluate_bruteforce(p, g, k) - refk)) < 1e-15
        assert np.max(np.abs(F.evaluate_windowed(p, g, k)[0] - refk)) < 1e-15


def test_identity_rotation_is_separable():
    g = F.Grid(12, 9, 7, x0=-2, y0=1, z0=3)
    mu, s = (3.2, 5.5, 6.1), (1.3, 2.1, 0.9)
    p = one(mu, (2.0, 0, 0, 0), s, -0.6)      # un-normalised identity
    gx = np.exp(-((g.x0 + np.arange(g.nx)) - mu[0]) ** 2 / (2 * s[0] ** 2))
    gy = np.exp(-((g.y0 + np.arange(g.ny)) - mu[1]) ** 2 / (2 * s[1] ** 2))
    gz = np.exp(-((g.z0 + np.arange(g.nz)) - mu[2]) ** 2 / (2 * s[2] ** 2))
    ref = -0.6 * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    assert np.max(np.abs(F.evaluate_bruteforce(p, g) - ref)) < 1e-15


def test_quarter_turn_about_z_swaps_x_and_y_scales():
    g = F.Grid(10, 10, 10)
    mu = (4.4, 4.9, 5.2)
    a = one(mu, (math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)), (1.1, 2.6, 1.9), 1.0)
    b = one(mu, (1, 0, 0, 0), (2.6, 1.1, 1.9), 1.0)
    assert np.max(np.abs(F.evaluate_bruteforce(a, g) - F.evaluate_bruteforce(b, g))) < 1e-14


def test_quaternion_sign_and_scale_invariance():
    g = F.Grid(8, 8, 8)
    p = S.random_params(3, 8, seed=3)
    base = F.evaluate_bruteforce(p, g, 3.0)
    for f in (-1.0, 0.37, 5.0):
        q = p.copy()
        q[3:7] *= f
        assert np.max(np.abs(F.evaluate_bruteforce(q, g, 3.0) - base)) < 1e-13


def test_matches_generator_formula():
    """The generator writes R as (w^2 - v.v)I + 2vv^T + 2w[v]x and m^2 as
    |S^-1 R^T d|^2; the oracle uses the Hamilton entries and d^T P d."""
    g = F.Grid(14, 13, 12)
    p = S.random_params(6, (14, 13, 12), seed=11, scale_range=(0.7, 3.0), unit_quat=False)
    ref = S.mixture_field(p, g.shape)
    assert np.max(np.abs(F.evaluate_bruteforce(p, g) - ref)) < 1e-12


def test_windowed_equals_bruteforce_and_permutation():
    g = F.Grid(16, 14, 12, x0=3, y0=-4, z0=1)
    p = S.random_params(25, (16, 14, 12), seed=5, scale_range=(0.6, 3.5), unit_quat=False)
    p[0] += g.x0
    p[1] += g.y0
    p[2] += g.z0
    for k in (1.5, 3.0, 5.0):
        vb = F.evaluate_bruteforce(p, g, k)
        vw, _ = F.evaluate_windowed(p, g, k)
        assert np.max(np.abs(vb - vw)) < 1e-13
        perm = np.random.default_rng(1).permutation(p.shape[1])
        vp, _ = F.evaluate_windowed(p[:, perm], g, k)
        assert np.max(np.abs(vp - vw)) < 1e-13


def test_truncation_pointwise_bound():
    g = F.Grid(20, 20, 20)
    p = S.random_params(12, 20, seed=9, scale_range=(1.0, 4.0))
    vinf = F.evaluate_bruteforce(p, g)
    for k, tail in ((3.0, 1.110900e-2), (5.0, 3.726653e-6)):
        assert abs(math.exp(-k * k / 2) - tail) / tail < 1e-6
        vk = F.evaluate_bruteforce(p, g, k)
        bound = math.exp(-k * k / 2) * np.sum(np.abs(p[10]))
        assert np.max(np.abs(vinf - vk)) <= bound * (1 + 1e-12)


@pytest.mark.parametrize("s,tol", [(1.0, 0.2), (1.5, 0.1), (2.5, 0.03), (4.0, 0.02)])
def test_truncation_integrated_tail(s, tol):
    k = 3.0
    n = int(2 * 8 * s) + 6
    g = F.Grid(n, n, n)
    c = 0.7
    mu = (n / 2 - 0.31, n / 2 + 0.17, n / 2 - 0.05)
    p = one(mu, (0.9, 0.2, -0.3, 0.1), (s, s * 1.1, s * 0.95), c)
    vinf = F.evaluate_bruteforce(p, g)
    vk, _ = F.evaluate_windowed(p, g, k)
    prod = s * (s * 1.1) * (s * 0.95)
    expect = c * (2 * math.pi) ** 1.5 * prod * q3_tail(k)
    assert abs(q3_tail(3.0) - 2.929089e-2) < 1e-8 and abs(q3_tail(5.0) - 1.544050e-5) < 1e-11
    assert abs(np.sum(vinf - vk) / expect - 1.0) < tol


@pytest.mark.parametrize("s", [1.0, 1.5, 2.3])
def test_poisson_lattice_sums(s):
    """sum_p G = (2 pi)^{3/2} det(Sigma)^{1/2} and sum_p G^2 = pi^{3/2} det^{1/2}
    on the integer lattice, up to exponentially small Poisson terms."""
    n = int(2 * 8 * s * 1.3) + 4
    g = F.Grid(n, n, n)
    sc = (s, 1.3 * s, 1.1 * s)
    p = one((n / 2 + 0.23, n / 2 - 0.41, n / 2 + 0.07), (0.3, -0.5, 0.6, 0.2), sc, 1.3)
    v = F.evaluate_bruteforce(p, g)
    prod = sc[0] * sc[1] * sc[2]
    assert abs(np.sum(v) / (1.3 * (2 * math.pi) ** 1.5 * prod) - 1) < 1e-8
    tol2 = 2e-5 if s < 1.5 else 1e-10
    assert abs(np.sum(v * v) / (1.3 ** 2 * math.pi ** 1.5 * prod) - 1) < tol2


def test_planted_solution_loss_equals_noise_energy():
    """With the 200 generating Gaussians, the untruncated residual is the noise:
    L = sum n^2 with n ~ N(0, 0.01^2) over 64^3 voxels."""
    f, gen = S.tiny_mixture(seed=0)
    g = F.Grid(64, 64, 64)
    v = F.evaluate_bruteforce(gen, g)
    L = float(np.sum((v - f.astype(np.float64)) ** 2))
    M = 64 ** 3
    mean, sd = M * 1e-4, 1e-4 * math.sqrt(2 * M)
    assert abs(mean - 26.2144) < 1e-9
    assert abs(L - mean) < 4 * sd, (L, mean, sd)


# --------------------------------------------------------------------------- gradient

def test_gradient_closed_forms_single_gaussian_zero_target():
    s = (1.8, 2.2, 1.6)
    c = 0.9
    n = 40
    g = F.Grid(n, n, n)
    p = one((19.6, 20.3, 19.9), (0.8, 0.1, -0.4, 0.3), s, c)
    k = 30.0   # effectively untruncated on this grid
    L, grad = F.loss_grad(p, np.zeros(g.shape), g, k)
    prod = s[0] * s[1] * s[2]
    expect = c * c * math.pi ** 1.5 * prod
    assert abs(L / expect - 1) < 1e-9
    assert abs(grad[10, 0] - 2 * L / c) < 1e-8 * L
    for j in range(3):
        assert abs(grad[7 + j, 0] - L) < 1e-8 * L
        assert abs(grad[j, 0]) < 1e-8 * L
    # rotating an anisotropic Gaussian does not change sum G^2 either
    assert np.max(np.abs(grad[3:7, 0])) < 1e-8 * L


def test_isotropic_quaternion_gradient_vanishes():
    g = F.Grid(12, 12, 12)
    p = one((5.3, 6.1, 5.7), (0.4, 0.5, -0.6, 0.2), (1.5, 1.5, 1.5), 0.7)
    fld = np.random.default_rng(0).uniform(size=g.shape)
    _, grad = F.loss_grad(p, fld, g, 3.0)
    assert np.max(np.abs(grad[3:7])) < 1e-12 * np.max(np.abs(grad))


def _min_boundary_gap(p, g, k):
    mu, _, _, _ = F.split(p)
    P = F.precision(p)
    zz, yy, xx = np.meshgrid(np.arange(g.nz) + g.z0, np.arange(g.ny) + g.y0,
                             np.arange(g.nx) + g.x0, indexing="ij")
    gap = np.inf
    for i in range(p.shape[1]):
        m2 = F._quad(P[i], xx - mu[i, 0], yy - mu[i, 1], zz - mu[i, 2])
        gap = min(gap, float(np.min(np.abs(m2 - k * k))))
    return gap


@pytest.mark.parametrize("k,seed", [(30.0, 0), (3.0, 1), (3.0, 2)])
def test_gradient_matches_central_differences(k, seed):
    g = F.Grid(11, 10, 12)
    p = S.random_params(4, (11, 10, 12), seed=seed, scale_range=(1.0, 2.5), unit_quat=False)
    fld = np.random.default_rng(seed + 50).uniform(-0.5, 1.0, size=g.shape)
    if k < 10:
        assert _min_boundary_gap(p, g, k) > 1e-4   # no voxel crosses the cut under FD
    L, grad = F.loss_grad(p, fld, g, k)
    fd = np.zeros_like(grad)
    for a in range(11):
        for i in range(p.shape[1]):
            h = 1e-6 * max(1.0, abs(p[a, i]))
            pp = p.copy()
            pm = p.copy()
            pp[a, i] += h
            pm[a, i] -= h
            fd[a, i] = (F.loss(pp, fld, g, k) - F.loss(pm, fld, g, k)) / (2 * h)
    scale = np.max(np.abs(grad), axis=1, keepdims=True)
    assert np.max(np.abs(fd - grad) / scale) < 1e-6


def test_quaternion_gradient_is_orthogonal_to_q():
    g = F.Grid(10, 11, 9)
    p = S.random_params(6, (10, 11, 9), seed=4, unit_quat=False)
    fld = np.random.default_rng(3).uniform(size=g.shape)
    _, grad = F.loss_grad(p, fld, g, 3.0)
    dots = np.sum(p[3:7] * grad[3:7], axis=0)
    assert np.max(np.abs(dots)) < 1e-12 * np.max(np.abs(grad[3:7]))


def test_gradient_permutes_with_primitives():
    g = F.Grid(10, 10, 10)
    p = S.random_params(7, 10, seed=8)
    fld = np.random.default_rng(2).uniform(size=g.shape)
    L, grad = F.loss_grad(p, fld, g, 3.0)
    perm = np.random.default_rng(4).permutation(7)
    L2, grad2 = F.loss_grad(p[:, perm], fld, g, 3.0)
    assert abs(L - L2) < 1e-12 * L
    assert np.max(np.abs(grad2 - grad[:, perm])) < 1e-12 * np.max(np.abs(grad))


# --------------------------------------------------------------------------- Adam

def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    p = rng.normal(size=(11, 5))
    gr = rng.normal(size=(11, 5))
    st = F.AdamState.zeros(5)
    out, _ = F.adam_update(p, gr, st, lr=1e-3)
    expect = p - 1e-3 * gr / (np.abs(gr) + 1e-8)
    assert np.max(np.abs(out - expect)) < 1e-15
    # |step| = lr |g| / (|g| + eps) differs from lr by at most lr eps / |g|
    assert np.max(np.abs(np.abs(out - p) - 1e-3)) <= 1e-3 * 1e-8 / np.min(np.abs(gr)) + 1e-15


def test_adam_two_steps_by_hand():
    p0, g1, g2, lr = 0.5, 0.2, -0.6, 0.01
    b1, b2, eps = 0.9, 0.999, 1e-8
    m1, v1 = 0.1 * g1, 0.001 * g1 * g1
    p1 = p0 - lr * (m1 / 0.1) / (math.sqrt(v1 / 0.001) + eps)
    m2, v2 = b1 * m1 + 0.1 * g2, b2 * v1 + 0.001 * g2 * g2
    p2 = p1 - lr * (m2 / (1 - b1 ** 2)) / (math.sqrt(v2 / (1 - b2 ** 2)) + eps)
    st = F.AdamState.zeros(1)
    x = np.full((11, 1), p0)
    x, _ = F.adam_update(x, np.full((11, 1), g1), st, lr)
    x, _ = F.adam_update(x, np.full((11, 1), g2), st, lr)
    assert st.t == 2
    assert np.max(np.abs(x - p2)) < 1e-15


def test_adam_clamp_counts_and_limits():
    p = np.zeros((11, 2))
    p[7:10] = [[-3.0, 0.0], [0.5, 4.0], [0.0, 0.0]]
    st = F.AdamState.zeros(2)
    out, n = F.adam_update(p, np.zeros((11, 2)), st, lr=0.0, ell_clamp=(-1.0, 2.0))
    assert n == 2
    assert out[7, 0] == -1.0 and out[8, 1] == 2.0


def test_refine_reduces_loss_on_mixture():
    g = F.Grid(16, 16, 16)
    gen = S.random_params(6, 16, seed=21, scale_range=(1.5, 3.0))
    fld = S.mixture_field(gen, g.shape)
    start = gen.copy()
    start[0:3] += np.random.default_rng(1).normal(0, 0.5, size=(3, 6))
    start[10] *= 0.7
    _, st, losses = F.refine(start, fld, g, 3.0, iters=30, lr=2e-2)
    assert st.t == 30
    assert losses[-1] < 0.5 * losses[0]


# --------------------------------------------------------------------------- metrics

def test_psnr_definition_and_sampled_estimate():
    assert F.psnr_from_mse(1e-2) == pytest.approx(20.0)
    rng = np.random.default_rng(0)
    a = rng.uniform(size=(64, 64, 64))
    b = a + rng.normal(0, 0.02, size=a.shape)
    full = float(np.mean((a - b) ** 2))
    samp = F.sampled_mse(a, b, 500_000, seed=123)
    # sampling std of the PSNR estimate for Gaussian residuals: 4.34 sqrt(2/n) dB
    sd_db = 10 / math.log(10) * math.sqrt(2.0 / 500_000)
    assert abs(F.psnr_from_mse(samp) - F.psnr_from_mse(full)) < 3 * sd_db


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_boundary_slack_bounds_the_effect_of_flipping_pairs(sign):
    """Moving the cut from k^2 to k^2 +- 0.9 band flips exactly the pairs the
    slack accounts for (those within band of the cut, on one side); the
    gradient change must stay within the slack."""
    grid = F.Grid(18, 16, 15)
    params = S.random_params(25, (18, 16, 15), seed=5, scale_range=(0.8, 3.0), unit_quat=False)
    field = np.random.default_rng(6).uniform(-1, 1, size=grid.shape)
    k, band = 3.0, 0.05
    slack, namb = F.boundary_slack(params, field, grid, k, band)
    assert namb > 10
    k2 = math.sqrt(k * k + sign * 0.9 * band)
    _, g0 = F.loss_grad(params, field, grid, k)
    _, g1 = F.loss_grad(params, field, grid, k2)
    diff = np.abs(g1 - g0)
    assert np.max(diff) > 0
    assert np.all(diff <= 1.01 * slack + 1e-12)
    # and the slack is not vacuous: same order as the change it bounds
    assert np.sum(slack) < 50 * np.sum(diff)


def test_absolute_gradient_bounds_the_gradient_and_matches_single_pair():
    """|dL/dtheta| <= sum of |per-pair terms| entrywise, with equality for c
    when every residual has one sign; on a one-voxel grid (a single pair per
    primitive) the absolute sum is |gradient| exactly."""
    grid = F.Grid(15, 13, 12)
    params = S.random_params(6, (15, 13, 12), seed=3, scale_range=(1.0, 3.0), unit_quat=False)
    field = np.random.default_rng(4).uniform(-1, 1, size=grid.shape)
    _, gr = F.loss_grad(params, field, grid, 3.0)
    ab = F.loss_grad_absolute(params, field, grid, 3.0)
    assert np.all(np.abs(gr) <= ab * (1 + 1e-12) + 1e-15)
    V, _ = F.evaluate_windowed(params, grid, 3.0)
    below = V - 5.0                        # target far above: every residual negative
    _, g2 = F.loss_grad(params, below, grid, 3.0)
    a2 = F.loss_grad_absolute(params, below, grid, 3.0)
    assert np.allclose(np.abs(g2[10]), a2[10], rtol=1e-12)
    one = F.Grid(1, 1, 1, 7, 6, 6)
    p1 = params.copy()
    p1[0:3] = np.array([[7.3], [6.2], [5.9]]) + np.random.default_rng(5).uniform(-0.5, 0.5, (3, 6))
    f1 = np.array([[[0.37]]])
    _, g1 = F.loss_grad(p1, f1, one, 3.0)
    a1 = F.loss_grad_absolute(p1, f1, one, 3.0)
    assert np.allclose(np.abs(g1), a1, rtol=1e-10, atol=1e-15)


def _one(mu, ell, q=(1.0, 0.0, 0.0, 0.0), c=1.0):
    p = np.zeros((11, 1))
    p[0:3, 0] = mu
    p[3:7, 0] = q
    p[7:10, 0] = ell
    p[10, 0] = c
    return p


def test_count_pairs_isotropic_ball_lattice_count():
    """An isotropic s = 1 Gaussian centred at (0.5, 0.5, 0.5) with k = 3: the
    in-support voxels are the integer points with |p - mu|^2 < 9, i.e. odd
    (u, v, w) = 2 (p - mu) with u^2 + v^2 + w^2 < 36.  With squares from
    {1, 9, 25}: (1,1,1) 8, (1,1,9) 24, (1,9,9) 24, (9,9,9) 8, (1,1,25) 24,
    (1,9,25) 48 sign/order patterns: 136 voxels, none on the boundary."""
    grid = F.Grid(20, 20, 20)
    p = _one((10.5, 10.5, 10.5), (0.0, 0.0, 0.0))
    assert F.count_pairs(p, grid, 3.0) == 136


def test_count_pairs_axis_aligned_ellipsoid_integer_count():
    """Scales (1, 2, 1/2) centred half-way between voxels: m^2 < 9 becomes
    4u^2 + v^2 + 16w^2 < 144 over odd integers (u, v, w), counted exactly in
    integers (the left side is 5 mod 8, so no point lies on the boundary)."""
    grid = F.Grid(24, 30, 16)
    p = _one((11.5, 14.5, 7.5), (0.0, math.log(2.0), -math.log(2.0)))
    odd = range(-31, 32, 2)
    ref = sum(1 for u in odd for v in odd for w in odd if 4 * u * u + v * v + 16 * w * w < 144)
    assert F.count_pairs(p, grid, 3.0) == ref
    # a grid that cuts the ellipsoid counts only what lies inside it
    cut = F.Grid(12, 30, 16)                       # x in [0, 11]: u = 2x - 23 <= -1
    ref_cut = sum(1 for u in odd for v in odd for w in odd
                  if u < 0 and 4 * u * u + v * v + 16 * w * w < 144)
    assert F.count_pairs(p, cut, 3.0) == ref_cut


@pytest.mark.parametrize("k", [2.0, 3.0, 5.0])
def test_count_pairs_equals_bruteforce_support_count(k):
    """For rotated anisotropic primitives (some hanging over the grid's faces)
    the windowed count equals the number of voxels where the brute-force
    truncated field of each primitive alone (c = 1) is nonzero."""
    grid = F.Grid(14, 11, 9, 2, -3, 1)
    params = S.random_params(6, (14, 11, 9), seed=int(k), scale_range=(0.5, 2.5),
                             unit_quat=False)
    params[0] += grid.x0 + np.array([-2.0, 0, 0, 3.0, 0, 0])
    params[1] += grid.y0
    params[2] += grid.z0
    params[10] = 1.0
    ref = 0
    for i in range(params.shape[1]):
        ref += int(np.count_nonzero(F.evaluate_bruteforce(params[:, i:i + 1], grid, k)))
    assert ref > 0
    assert F.count_pairs(params, grid, k) == ref


def test_count_pairs_cut_is_strict_on_lattice_boundary_points():
    """Centred on a voxel with s = 1 and k = 3, m^2 = |p - mu|^2 is an exact
    integer; the voxels with |p - mu|^2 < 9 number sum_{n < 9} r3(n) =
    1 + 6 + 12 + 8 + 6 + 24 + 24 + 0 + 12 = 93 (r3(n): representations of n as a
    sum of three squares), and the 30 voxels with |p - mu|^2 = 9 ((3,0,0) and
    (2,2,1) up to sign and order) lie on the cut and are excluded."""
    grid = F.Grid(15, 15, 15)
    p = _one((7.0, 7.0, 7.0), (0.0, 0.0, 0.0))
    assert F.count_pairs(p, grid, 3.0) == 93
    V = F.evaluate_bruteforce(p, grid, 3.0)
    assert np.count_nonzero(V) == 93


def test_bruteforce_gradient_equals_windowed_and_splits_over_primitives():
    """Visiting every voxel adds only exact zeros outside each support box, so
    the brute-force loss and gradient equal the windowed ones (up to the
    summation order of the sums); and with the residual held fixed each
    primitive's gradient depends only on its own pairs."""
    grid = F.Grid(13, 11, 9, 1, -2, 0)
    params = S.random_params(7, (13, 11, 9), seed=5, scale_range=(0.6, 2.5), unit_quat=False)
    params[0] += grid.x0 + np.array([-2.0, 0, 0, 3.0, 0, 0, 0])
    params[1] += grid.y0
    field = np.random.default_rng(6).uniform(size=grid.shape)
    L, g = F.loss_grad(params, field, grid, 3.0)
    Lb, gb = F.loss_grad_bruteforce(params, field, grid, 3.0)
    assert abs(Lb - L) <= 1e-13 * L
    assert np.allclose(gb, g, rtol=1e-12, atol=1e-13 * np.max(np.abs(g)))
    V, _ = F.evaluate_windowed(params, grid, 3.0)
    r = 2.0 * (V - field)
    ga, _ = F.grad_from_residual(params[:, :3], r, grid, 3.0)
    gz, _ = F.grad_from_residual(params[:, 3:], r, grid, 3.0)
    assert np.array_equal(np.concatenate([ga, gz], axis=1), g)
