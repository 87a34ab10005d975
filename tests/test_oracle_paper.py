"""Pins for the oracle of the paper's own training loop (CPU only).

* The ratio field reduces to a scaled sum field where the density stays under
  the floor rho0, and to the attribute itself where a single primitive's
  density exceeds it (eq:field).
* Below the floor, value loss and gradient equal the sum-model oracle's
  (``oracle.field``, pinned separately) with c = w a / rho0.
* Every objective term's analytic gradient agrees with central differences.
* Trilinear interpolation, the stratified sampler (class structure, jitter,
  determinism), Adam's first step, the conversion from an allocation.
"""
import math

import numpy as np
import pytest

from oracle import field as F
from oracle import paper as Pp
from synth import fields as S


def _theta(n, extent, seed, scale_range=(1.0, 3.0), w_range=(0.2, 0.8)):
    p = S.random_params(n, extent, seed=seed, scale_range=scale_range, unit_quat=False)
    rng = np.random.default_rng(seed + 100)
    th = np.zeros((12, n))
    th[0:10] = p[0:10]
    th[10] = rng.uniform(0.1, 0.9, n)
    w = rng.uniform(*w_range, n)
    th[11] = np.log(w / (1 - w))
    return th


def test_single_primitive_closed_forms():
    th = np.zeros((12, 1))
    th[0:3, 0] = (5.0, 5.0, 5.0)
    th[3, 0] = 1.0
    th[7:10, 0] = math.log(2.0)
    th[10, 0] = 0.7
    th[11, 0] = math.log(0.5 / 0.5)        # w = 0.5
    pts = np.array([[5.0, 5.0, 5.0], [6.0, 5.5, 4.0], [5.0, 5.0, 12.0], [5.0, 5.0, 15.5]])
    Vt, num, den = Pp.field_at(th, pts, k=5.0, rho0=0.05)
    G = np.exp(-0.5 * np.sum((pts - 5.0) ** 2, axis=1) / 4.0)
    G[np.sum((pts - 5.0) ** 2, axis=1) / 4.0 >= 25.0] = 0.0
    assert np.allclose(den, 0.5 * G, rtol=1e-15, atol=0)
    for s in range(4):
        expect = 0.7 if 0.5 * G[s] > 0.05 else 0.7 * 0.5 * G[s] / 0.05
        assert abs(Vt[s] - expect) < 1e-15
    assert Vt[3] == 0.0                         # beyond 5 sigma


def test_below_the_floor_equals_the_sum_model():
    grid = F.Grid(14, 12, 11)
    th = _theta(6, (14, 12, 11), seed=3, w_range=(0.004, 0.008))
    field = np.random.default_rng(4).uniform(0.1, 0.9, size=grid.shape)
    zz, yy, xx = np.meshgrid(np.arange(11), np.arange(12), np.arange(14), indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.float64)
    vals = field.ravel()
    opt = Pp.Options(k=3.0, lam_rho=0.0, lam_sm=0.0, lam_anc=0.0, lam_aniso=0.0, lam_cap=0.0)
    _, _, den = Pp.field_at(th, pts, opt.k, opt.rho0)
    assert den.max() < opt.rho0
    w = Pp.sigmoid(th[11])
    p11 = np.zeros((11, 6))
    p11[0:10] = th[0:10]
    p11[10] = w * th[10] / opt.rho0
    L, parts = Pp.objective(th, field, grid, pts, pts, vals, opt)
    Ls, gs = F.loss_grad(p11, field, grid, opt.k)
    assert abs(parts[0] - Ls) <= 1e-12 * Ls
    g = Pp.objective_grad(th, field, grid, pts, pts, vals, opt)
    assert np.allclose(g[0:10], gs[0:10], rtol=1e-10, atol=1e-12 * np.abs(gs).max())
    assert np.allclose(g[10], gs[10] * w / opt.rho0, rtol=1e-10, atol=1e-15)
    assert np.allclose(g[11], gs[10] * th[10] * w * (1 - w) / opt.rho0, rtol=1e-10, atol=1e-15)


def _kink_free(th, pts, partners, vals, opt, h):
    """True if no finite-difference step can cross a kink of the objective."""
    mu, _, ell, _, _ = Pp.split(th)
    _, P, _, _, _ = Pp._geometry(th)
    for X in (pts, partners):
        _, _, den = Pp.field_at(th, X, opt.k, opt.rho0)
        if np.min(np.abs(den - opt.rho0)) < 1e-3:
            return False
        for i in range(mu.shape[0]):
            d = X - mu[i]
            m2 = np.einsum("sj,jk,sk->s", d, P[i], d)
            if np.min(np.abs(m2 - opt.k ** 2)) < 1e-3:
                return False
    spread = ell.max(axis=1) - ell.min(axis=1) - math.log(opt.aniso_max)
    srt = np.sort(ell, axis=1)
    return (np.min(np.abs(spread)) > 1e-4 and np.min(np.abs(ell - opt.ell_hi)) > 1e-4
            and np.min(np.abs(ell - opt.ell_lo)) > 1e-4 and np.min(np.diff(srt, axis=1)) > 1e-4
            and np.all(np.abs(np.asarray(vals) - opt.v_occ) > 1e-6))


def test_objective_gradient_matches_central_differences():
    grid = F.Grid(16, 15, 14)
    th = _theta(5, (16, 15, 14), seed=7, scale_range=(1.2, 3.0))
    th[7:10, 0] = np.log([0.6, 2.0, 3.5])     # outside 3:1 and below ell_lo: both regulisers on
    th[7:10, 1] = np.log([1.1, 1.3, 9.0])
    field = np.random.default_rng(8).uniform(0.0, 1.0, size=grid.shape)
    opt = Pp.Options(k=3.0, rho0=0.05, lam_rho=0.3, lam_sm=0.2, lam_anc=0.05, lam_aniso=0.7,
                     lam_cap=0.9, ell_lo=math.log(0.8), ell_hi=math.log(6.0))
    pts, partners, vals = Pp.sample_points(field, grid, 80, seed=11, it=0, opt=opt)
    h = 1e-6
    assert _kink_free(th, pts, partners, vals, opt, h)
    g = Pp.objective_grad(th, field, grid, pts, partners, vals, opt)
    for i in range(th.shape[1]):
        for j in range(12):
            hh = h * max(1.0, abs(th[j, i]))
            tp, tm = th.copy(), th.copy()
            tp[j, i] += hh
            tm[j, i] -= hh
            fd = (Pp.objective(tp, field, grid, pts, partners, vals, opt)[0]
                  - Pp.objective(tm, field, grid, pts, partners, vals, opt)[0]) / (2 * hh)
            # the anchor reference V(mu) is held fixed in the gradient: remove its
            # finite-difference share along mu
            if j < 3:
                mu = th[0:3, i].copy()
                dmu = np.zeros(3)
                dmu[j] = hh
                vp = Pp.trilinear(field, grid, (mu + dmu)[None])[0]
                vm = Pp.trilinear(field, grid, (mu - dmu)[None])[0]
                a = th[10, i]
                fd -= opt.lam_anc * ((a - vp) ** 2 - (a - vm) ** 2) / (2 * hh)
            assert abs(fd - g[j, i]) <= 1e-6 * max(1.0, abs(fd)), (i, j, fd, g[j, i])


def test_trilinear_interpolation():
    grid = F.Grid(7, 6, 5, 2, -1, 3)
    zz, yy, xx = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    lin = 0.3 * xx - 0.7 * yy + 1.1 * zz + 0.25
    rng = np.random.default_rng(0)
    pts = np.stack([rng.uniform(2, 8, 50), rng.uniform(-1, 4, 50), rng.uniform(3, 7, 50)], axis=1)
    got = Pp.trilinear(lin, grid, pts)
    ref = 0.3 * (pts[:, 0] - 2) - 0.7 * (pts[:, 1] + 1) + 1.1 * (pts[:, 2] - 3) + 0.25
    assert np.allclose(got, ref, atol=1e-12)
    f = rng.uniform(size=grid.shape)
    centers = np.array([[2 + 3, -1 + 2, 3 + 4], [2, -1, 3], [8, 4, 7]], dtype=np.float64)
    assert np.allclose(Pp.trilinear(f, grid, centers), [f[4, 2, 3], f[0, 0, 0], f[4, 5, 6]])
    assert Pp.trilinear(f, grid, np.array([[-50.0, -50.0, -50.0]]))[0] == f[0, 0, 0]


def test_sampler_classes_jitter_and_determinism():
    grid = F.Grid(20, 18, 16)
    field = np.zeros(grid.shape, dtype=np.float32)
    field[4:9, 5:10, 6:12] = 0.8            # high class
    field[10:14, 2:16, 3:17] = 0.2          # mid class
    opt = Pp.Options()
    n = 200
    pts, partners, vals = Pp.sample_points(field, grid, n, seed=5, it=3, opt=opt)
    n_hi, n_mid, n_uni = Pp.class_counts(n, 1, 1, opt)
    assert (n_hi, n_mid, n_uni) == (70, 80, 50)
    vox = np.rint(pts).astype(int)
    cls = field[vox[:, 2], vox[:, 1], vox[:, 0]]
    assert np.all(cls[:n_hi] > 0.4)
    assert np.all((cls[n_hi:n_hi + n_mid] > 0.02) & (cls[n_hi:n_hi + n_mid] <= 0.4))
    assert np.all(np.abs(pts - vox) <= 0.5) and np.all(np.abs(partners - pts) <= 0.5)
    assert np.allclose(vals, Pp.trilinear(field, grid, pts))
    p2, q2, v2 = Pp.sample_points(field, grid, n, seed=5, it=3, opt=opt)
    assert np.array_equal(p2, pts) and np.array_equal(q2, partners)
    p3, _, _ = Pp.sample_points(field, grid, n, seed=5, it=4, opt=opt)
    assert not np.array_equal(p3, pts)
    # no high voxels: their share goes to the uniform class
    assert Pp.class_counts(n, 0, 10, opt) == (0, 80, 120)


def test_adam_first_step_and_from_allocation():
    th = np.ones((12, 3))
    g = np.linspace(-1, 1, 36).reshape(12, 3)
    g[g == 0] = 0.5
    out, m, v = Pp.adam(th, g, np.zeros_like(th), np.zeros_like(th), 1, lr=8e-3)
    assert np.allclose(out, th - 8e-3 * np.sign(g), atol=1e-9)
    p11 = np.arange(33, dtype=np.float64).reshape(11, 3)
    t12 = Pp.from_allocation(p11, kappa=2.0, w0=0.1)
    assert np.array_equal(t12[0:10], p11[0:10])
    assert np.allclose(t12[10], p11[10] / 2.0)
    assert np.allclose(Pp.sigmoid(t12[11]), 0.1)
    assert Pp.lam_sm_at(0, 11, 1.0, 0.0) == 1.0 and Pp.lam_sm_at(10, 11, 1.0, 0.0) == 0.0
