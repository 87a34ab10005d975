"""Oracle: the paper's own training loop (Sec. III-C eq:field, Sec. III-F).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  NumPy float64, plain
loops over primitives and sample points.

Each primitive carries 12 numbers (rows of ``theta``): centre mu (3), raw
quaternion q (4, scalar first), log-scales ell (3), scalar attribute a, and
the weight logit b with w = sigmoid(b) (Sec. III-C: log-scales, normalised
quaternion, sigmoid-activated logits).  The field is the density-normalised
kernel regression of eq:field,

    Vt(p) = sum_i w_i a_i G_i(p) / max(sum_i w_i G_i(p), rho0),   rho0 = 0.05,

with G_i truncated where m^2 >= k^2 (k = 5 in the paper).  Training draws
3,072 stratified, jittered sample points per iteration (35 % from voxels with
V > 0.4, 40 % from occupied mid-range voxels, 25 % uniform; Sec. III-F and
Table tab:training-config) and minimises

    L = L_val + lam_rho L_rho + lam_sm L_sm + lam_anc L_anc
        + lam_aniso L_aniso + lam_cap L_cap.

Readings of what the paper leaves open (each is a knob):

* Sampling: class members are picked uniformly with replacement from the
  class's voxels in ascending index order, voxel j = floor(u n_class) with u
  from the counter generator of ``oracle.alloc`` (streams below); a class
  with no voxels gives its share to the uniform class.  Jitter is
  U[-1/2, 1/2]^3 per point.  "Mid-range" is v_occ < V <= v_hi.  The value at
  a jittered point is the trilinear interpolation of the volume (clamped to
  the grid).
* L_val = sum over samples with V > 0.02 of (Vt - V)^2 (Sec. III-F's
  indicator and squared norm).
* L_rho = sum over the same samples of (rho - 1)^2 (a unit density target
  over occupied space, both directions).
* L_sm = sum over samples of (rho(p) - rho(p'))^2 with p' = p + U[-1/2, 1/2]^3
  (a nearby jittered partner per sample); lam_sm anneals linearly from
  lam_sm_start to lam_sm_end over the schedule.
* L_anc = sum_i (a_i - V(mu_i))^2 with V(mu_i) trilinear and held fixed
  (no gradient into mu).
* L_aniso = sum_i relu((max_j ell_ij - min_j ell_ij) - ln 3)^2 (the 3:1
  elongation bound).
* L_cap = sum_ij relu(ell_ij - ell_hi)^2 + relu(ell_lo - ell_ij)^2 with the
  range [ell_lo, ell_hi] taken from the initialisation.
* Derivative of max(den, rho0): the density term passes gradient only where
  den > rho0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import alloc as A
from . import field as F

NPARAM = 12
STREAM_PICK = 20         # class member of sample s
STREAM_JIT = 21          # + axis: jitter of sample s
STREAM_PARTNER = 24      # + axis: offset of its smoothness partner


@dataclass
class Options:
    k: float = 5.0
    rho0: float = 0.05
    samples: int = 3072
    frac_hi: float = 0.35
    frac_mid: float = 0.40
    v_hi: float = 0.4
    v_occ: float = 0.02
    lam_rho: float = 0.1
    lam_sm: float = 0.1
    lam_anc: float = 0.01
    lam_aniso: float = 1.0
    lam_cap: float = 1.0
    aniso_max: float = 3.0
    ell_lo: float = math.log(0.25)
    ell_hi: float = math.log(64.0)


def split(theta):
    t = np.asarray(theta, dtype=np.float64)
    assert t.ndim == 2 and t.shape[0] == NPARAM, t.shape
    return t[0:3].T, t[3:7].T, t[7:10].T, t[10], t[11]


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-np.asarray(x, dtype=np.float64)))


def _geometry(theta):
    """(R, P) of every primitive through the sum-model helpers (rows 0-9 agree)."""
    t11 = np.asarray(theta, dtype=np.float64)[0:11].copy()
    qn, qnorm, qok = F.normalize_quat(t11[3:7].T)
    return F.rotation(qn), F.precision(t11), qn, qnorm, qok


def kernels(theta, pts, k):
    """G[i, s] = exp(-m^2 / 2) where m^2 < k^2, else 0 (every pair)."""
    mu, _, _, _, _ = split(theta)
    _, P, _, _, _ = _geometry(theta)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    G = np.zeros((mu.shape[0], pts.shape[0]))
    for i in range(mu.shape[0]):
        d = pts - mu[i]
        m2 = np.einsum("sj,jk,sk->s", d, P[i], d)
        G[i] = np.where(m2 < k * k, np.exp(-0.5 * m2), 0.0)
    return G


def field_at(theta, pts, k, rho0):
    """(Vt, num, den) at the points (eq:field)."""
    _, _, _, a, b = split(theta)
    w = sigmoid(b)
    G = kernels(theta, pts, k)
    num = (w * a) @ G
    den = w @ G
    return num / np.maximum(den, rho0), num, den


def trilinear(field, grid: F.Grid, pts):
    """Trilinear interpolation of the volume at world points, clamped to the grid."""
    v = np.asarray(field, dtype=np.float64).reshape(grid.shape)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    dims = (grid.nx, grid.ny, grid.nz)
    org = (grid.x0, grid.y0, grid.z0)
    for s, p in enumerate(pts):
        lo, fr = [], []
        for j in range(3):
            x = min(max(p[j] - org[j], 0.0), dims[j] - 1.0)
            i0 = min(int(math.floor(x)), dims[j] - 2) if dims[j] > 1 else 0
            lo.append(i0)
            fr.append(x - i0 if dims[j] > 1 else 0.0)
        acc = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    ix = min(lo[0] + dx, dims[0] - 1)
                    iy = min(lo[1] + dy, dims[1] - 1)
                    iz = min(lo[2] + dz, dims[2] - 1)
                    wgt = ((fr[0] if dx else 1 - fr[0]) * (fr[1] if dy else 1 - fr[1])
                           * (fr[2] if dz else 1 - fr[2]))
                    acc += wgt * v[iz, iy, ix]
        out[s] = acc
    return out


def class_counts(n, n_hi_vox, n_mid_vox, opt: Options):
    """Samples per class (hi, mid, uniform)."""
    n_hi = int(math.floor(opt.frac_hi * n + 0.5)) if n_hi_vox else 0
    n_mid = int(math.floor(opt.frac_mid * n + 0.5)) if n_mid_vox else 0
    return n_hi, n_mid, n - n_hi - n_mid


def sample_points(field, grid: F.Grid, n, seed, it, opt: Options):
    """(points [n, 3], partners [n, 3], values [n]) of iteration ``it``.

    Samples 0 .. n_hi-1 come from the high class, then the mid class, then the
    uniform class; sample s uses counter index it * n + s.
    """
    v = np.asarray(field, dtype=np.float32).ravel()
    hi = np.nonzero(v > np.float32(opt.v_hi))[0]
    mid = np.nonzero((v > np.float32(opt.v_occ)) & (v <= np.float32(opt.v_hi)))[0]
    n_hi, n_mid, _ = class_counts(n, hi.size, mid.size, opt)
    pts = np.zeros((n, 3))
    partners = np.zeros((n, 3))
    M = v.size
    for s in range(n):
        idx = np.uint64(it) * np.uint64(n) + np.uint64(s)
        u = float(A.uniform01(seed, STREAM_PICK, idx))
        if s < n_hi:
            vox = int(hi[min(int(math.floor(u * hi.size)), hi.size - 1)])
        elif s < n_hi + n_mid:
            vox = int(mid[min(int(math.floor(u * mid.size)), mid.size - 1)])
        else:
            vox = min(int(math.floor(u * M)), M - 1)
        ix = vox % grid.nx
        iy = (vox // grid.nx) % grid.ny
        iz = vox // (grid.nx * grid.ny)
        base = (grid.x0 + ix, grid.y0 + iy, grid.z0 + iz)
        for j in range(3):
            pts[s, j] = base[j] + float(A.uniform01(seed, STREAM_JIT + j, idx)) - 0.5
            partners[s, j] = pts[s, j] + float(A.uniform01(seed, STREAM_PARTNER + j, idx)) - 0.5
    return pts, partners, trilinear(field, grid, pts)


def objective(theta, field, grid: F.Grid, pts, partners, vals, opt: Options):
    """(L, parts) with parts = (L_val, L_rho, L_sm, L_anc, L_aniso, L_cap)."""
    mu, _, ell, a, _ = split(theta)
    Vt, _, den = field_at(theta, pts, opt.k, opt.rho0)
    _, _, den2 = field_at(theta, partners, opt.k, opt.rho0)
    occ = np.asarray(vals) > opt.v_occ
    L_val = float(np.sum(np.where(occ, (Vt - vals) ** 2, 0.0)))
    L_rho = float(np.sum(np.where(occ, (den - 1.0) ** 2, 0.0)))
    L_sm = float(np.sum((den - den2) ** 2))
    a_ref = trilinear(field, grid, mu)
    L_anc = float(np.sum((a - a_ref) ** 2))
    spread = ell.max(axis=1) - ell.min(axis=1) - math.log(opt.aniso_max)
    L_aniso = float(np.sum(np.maximum(spread, 0.0) ** 2))
    L_cap = float(np.sum(np.maximum(ell - opt.ell_hi, 0.0) ** 2
                         + np.maximum(opt.ell_lo - ell, 0.0) ** 2))
    parts = (L_val, L_rho, L_sm, L_anc, L_aniso, L_cap)
    L = (L_val + opt.lam_rho * L_rho + opt.lam_sm * L_sm + opt.lam_anc * L_anc
         + opt.lam_aniso * L_aniso + opt.lam_cap * L_cap)
    return L, parts


def _geom_grad(g, d, P, R, ell, qn, qnorm, qok):
    """d/d(mu, q, ell) of sum_s g_s G(p_s) through G, from the weighted
    moments of d = p - mu (the same contractions as ``oracle.field.loss_grad``)."""
    out = np.zeros(10)
    Sgd = (g[:, None] * d).sum(axis=0)
    D = np.einsum("s,sj,sk->jk", g, d, d)
    out[0:3] = P @ Sgd
    si2 = np.exp(-2.0 * ell)
    out[7:10] = si2 * np.diag(R.T @ D @ R)
    if qok:
        dR = -D @ R @ np.diag(si2)
        dRq = F.rotation_partials(qn)
        dqn = np.array([np.sum(dR * dRq[c]) for c in range(4)])
        out[3:7] = (np.eye(4) - np.outer(qn, qn)) @ dqn / qnorm
    return out


def objective_grad(theta, field, grid: F.Grid, pts, partners, vals, opt: Options):
    """dL/dtheta (12, N) of ``objective`` (quotient rule; see the module notes)."""
    mu, _, ell, a, b = split(theta)
    R, P, qn, qnorm, qok = _geometry(theta)
    w = sigmoid(b)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    partners = np.asarray(partners, dtype=np.float64).reshape(-1, 3)
    Vt, _, den = field_at(theta, pts, opt.k, opt.rho0)
    _, _, den2 = field_at(theta, partners, opt.k, opt.rho0)
    occ = np.asarray(vals) > opt.v_occ
    u = np.where(occ, 2.0 * (Vt - vals), 0.0)                  # dL/dVt
    v = (np.where(occ, 2.0 * opt.lam_rho * (den - 1.0), 0.0)
         + 2.0 * opt.lam_sm * (den - den2))                     # dL/dden (main points)
    v2 = -2.0 * opt.lam_sm * (den - den2)                       # dL/dden (partners)
    D = np.maximum(den, opt.rho0)
    alpha = u / D                                               # on d(w a G)
    beta = v - np.where(den > opt.rho0, u * Vt / D, 0.0)        # on d(w G)
    G1 = kernels(theta, pts, opt.k)
    G2 = kernels(theta, partners, opt.k)
    N = mu.shape[0]
    grad = np.zeros((NPARAM, N))
    for i in range(N):
        coef1 = (alpha * a[i] + beta) * w[i]      # d/dG_i(p_s), main points
        coef2 = v2 * w[i]                         # partners
        g = np.concatenate([coef1 * G1[i], coef2 * G2[i]])
        d = np.concatenate([pts, partners]) - mu[i]
        grad[0:10, i] = _geom_grad(g, d, P[i], R[i], ell[i], qn[i], qnorm[i], qok[i])
        grad[10, i] = np.sum(alpha * w[i] * G1[i])
        grad[11, i] = (np.sum((alpha * a[i] + beta) * G1[i]) + np.sum(v2 * G2[i])) \
            * w[i] * (1.0 - w[i])
    # regularisers
    a_ref = trilinear(field, grid, mu)
    grad[10] += 2.0 * opt.lam_anc * (a - a_ref)
    for i in range(N):
        jmax = int(np.argmax(ell[i]))
        jmin = int(np.argmin(ell[i]))
        e = ell[i, jmax] - ell[i, jmin] - math.log(opt.aniso_max)
        if e > 0:
            grad[7 + jmax, i] += 2.0 * opt.lam_aniso * e
            grad[7 + jmin, i] -= 2.0 * opt.lam_aniso * e
        for j in range(3):
            if ell[i, j] > opt.ell_hi:
                grad[7 + j, i] += 2.0 * opt.lam_cap * (ell[i, j] - opt.ell_hi)
            if ell[i, j] < opt.ell_lo:
                grad[7 + j, i] -= 2.0 * opt.lam_cap * (opt.ell_lo - ell[i, j])
    return grad


def lam_sm_at(it, iters, start, end):
    """Linear anneal of the smoothness weight over a schedule of ``iters``."""
    if iters <= 1:
        return start
    return start + (end - start) * it / (iters - 1)


def adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step on all 12 rows (t is the new step count)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    th = theta - lr * (m / (1 - beta1 ** t)) / (np.sqrt(v / (1 - beta2 ** t)) + eps)
    return th, m, v


def from_allocation(params11, kappa, w0):
    """12-row set from an allocated sum-model set: a = c / kappa (the volume's
    value at the seed), weight logit of w0 (uniform low initial weights)."""
    p = np.asarray(params11, dtype=np.float64)
    out = np.zeros((NPARAM, p.shape[1]))
    out[0:10] = p[0:10]
    out[10] = p[10] / kappa
    out[11] = math.log(w0 / (1.0 - w0))
    return out
