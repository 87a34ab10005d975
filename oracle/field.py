"""Oracle: truncated Gaussian field, sum-of-squares loss, analytic gradient, Adam.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  float64 NumPy.

What is computed (paper Sec. III-C, eq:field and the sentence after it, read for
an unnormalised weighted sum with one scalar weight per primitive):

    V_k(p) = sum_i c_i * G_i(p) * [m_i(p)^2 < k^2]
    G_i(p) = exp(-m_i(p)^2 / 2),  m_i(p)^2 = (p - mu_i)^T Sigma_i^{-1} (p - mu_i)
    Sigma_i = R(q_i) S_i S_i^T R(q_i)^T,   S_i = diag(exp(l_i))

* Parameters per primitive (11): mu (3), raw quaternion q = (w, x, y, z)
  (scalar first, Hamilton; normalised inside the forward pass as the paper's
  "normalized quaternion", Sec. III-C), log-scales l (3), weight c (1).
* Truncation is the hard cut of Sec. III-C ("squared Mahalanobis distance
  below" k^2, strict), with k a parameter (the paper uses 5, the workloads
  here use 3).
* Coordinates are voxel-index coordinates (Sec. III-B): voxel (i, j, k) of a
  grid sits at (x0 + i, y0 + j, z0 + k).  Arrays are indexed [z, y, x]
  (x fastest in memory).
* Loss: L = sum_p (V_k(p) - V(p))^2 over every voxel of the grid, the squared
  norm of the value term of Sec. III-F without its occupancy mask.
  MSE = L / M and PSNR = 10 log10(1 / MSE) (Sec. IV-C).
* Gradient: the derivative of L with the truncation indicator held fixed (the
  truncated evaluator "preserves ... its gradients", Sec. III-G).
* Optimiser: Adam (Kingma and Ba, cited in Sec. III-F), bias corrected.

Parameter arrays are float64 of shape (11, N) in the order
mu_x, mu_y, mu_z, q_w, q_x, q_y, q_z, l_x, l_y, l_z, c.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

NPARAM = 11


@dataclass(frozen=True)
class Grid:
    """A regular voxel grid in voxel-index coordinates (Sec. III-B)."""

    nx: int
    ny: int
    nz: int
    x0: int = 0
    y0: int = 0
    z0: int = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def size(self):
        return self.nx * self.ny * self.nz


# ----------------------------------------------------------------------------
# Primitive geometry
# ----------------------------------------------------------------------------

def split(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.ndim == 2 and p.shape[0] == NPARAM, p.shape
    mu = p[0:3].T.copy()          # (N, 3)
    q = p[3:7].T.copy()           # (N, 4)
    ell = p[7:10].T.copy()        # (N, 3)
    c = p[10].copy()              # (N,)
    return mu, q, ell, c


def normalize_quat(q):
    """Unit quaternion and its norm; a (near) zero quaternion is the identity."""
    q = np.asarray(q, dtype=np.float64)
    n = np.sqrt(np.sum(q * q, axis=-1))
    qn = np.zeros_like(q)
    ok = n >= 1e-12
    qn[ok] = q[ok] / n[ok, None]
    qn[~ok] = np.array([1.0, 0.0, 0.0, 0.0])
    return qn, n, ok


def rotation(qn):
    """Rotation matrix of unit quaternions (w, x, y, z), Hamilton convention."""
    w, x, y, z = qn[..., 0], qn[..., 1], qn[..., 2], qn[..., 3]
    R = np.empty(qn.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rotation_partials(qn):
    """dR/dw, dR/dx, dR/dy, dR/dz for one unit quaternion: array (4, 3, 3)."""
    w, x, y, z = qn
    dw = np.array([[0, -2 * z, 2 * y], [2 * z, 0, -2 * x], [-2 * y, 2 * x, 0]])
    dx = np.array([[0, 2 * y, 2 * z], [2 * y, -4 * x, -2 * w], [2 * z, 2 * w, -4 * x]])
    dy = np.array([[-4 * y, 2 * x, 2 * w], [2 * x, 0, 2 * z], [-2 * w, 2 * z, -4 * y]])
    dz = np.array([[-4 * z, -2 * w, 2 * x], [2 * w, -4 * z, 2 * y], [2 * x, 2 * y, 0]])
    return np.stack([dw, dx, dy, dz]).astype(np.float64)


def covariance(params):
    """Sigma_i = R S S^T R^T for every primitive: (N, 3, 3)."""
    _, q, ell, _ = split(params)
    qn, _, _ = normalize_quat(q)
    R = rotation(qn)
    s2 = np.exp(2.0 * ell)
    return np.einsum("nij,nj,nkj->nik", R, s2, R)


def precision(params):
    """Sigma_i^{-1} = R S^{-2} R^T for every primitive: (N, 3, 3)."""
    _, q, ell, _ = split(params)
    qn, _, _ = normalize_quat(q)
    R = rotation(qn)
    si2 = np.exp(-2.0 * ell)
    return np.einsum("nij,nj,nkj->nik", R, si2, R)


def support_box(mu, cov, k, grid: Grid):
    """Index ranges (inclusive) of voxels that can satisfy m^2 < k^2.

    |d_j| >= k sqrt(Sigma_jj) implies m^2 >= k^2 (Cauchy-Schwarz), so every
    in-support voxel lies in this box.  Returns None when the box is empty.
    """
    lo = (grid.x0, grid.y0, grid.z0)
    n = (grid.nx, grid.ny, grid.nz)
    out = []
    for j in range(3):
        h = k * math.sqrt(cov[j, j])
        a = max(0, math.ceil(mu[j] - h - lo[j]))
        b = min(n[j] - 1, math.floor(mu[j] + h - lo[j]))
        if a > b:
            return None
        out.append((a, b))
    return out


def _box_offsets(box, mu, grid: Grid):
    (ia, ib), (ja, jb), (ka, kb) = box
    xs = grid.x0 + np.arange(ia, ib + 1) - mu[0]
    ys = grid.y0 + np.arange(ja, jb + 1) - mu[1]
    zs = grid.z0 + np.arange(ka, kb + 1) - mu[2]
    dz, dy, dx = np.meshgrid(zs, ys, xs, indexing="ij")
    return dx, dy, dz


def _quad(P, dx, dy, dz):
    return (P[0, 0] * dx * dx + P[1, 1] * dy * dy + P[2, 2] * dz * dz
            + 2.0 * (P[0, 1] * dx * dy + P[0, 2] * dx * dz + P[1, 2] * dy * dz))


# ----------------------------------------------------------------------------
# Evaluation
# ----------------------------------------------------------------------------

def evaluate_bruteforce(params, grid: Grid, k=None):
    """V_k on every voxel by visiting every (primitive, voxel) pair.

    k=None drops the truncation (the untruncated field V_inf).
    """
    mu, _, _, c = split(params)
    P = precision(params)
    zz, yy, xx = np.meshgrid(grid.z0 + np.arange(grid.nz), grid.y0 + np.arange(grid.ny),
                             grid.x0 + np.arange(grid.nx), indexing="ij")
    out = np.zeros(grid.shape)
    for i in range(mu.shape[0]):
        m2 = _quad(P[i], xx - mu[i, 0], yy - mu[i, 1], zz - mu[i, 2])
        g = np.exp(-0.5 * m2)
        if k is not None:
            g = np.where(m2 < k * k, g, 0.0)
        out += c[i] * g
    return out


def evaluate_windowed(params, grid: Grid, k, band=0.0):
    """V_k on every voxel, visiting only each primitive's support box.

    Identical to ``evaluate_bruteforce`` for finite k (see ``support_box``).
    With band > 0 also returns (V_lo, V_hi, n_ambiguous): pairs whose m^2 lies
    within ``band`` of k^2 are excluded from V_lo and included in V_hi, and
    counted, so that a float32 evaluator whose boundary decision differs from
    float64 can be bracketed.  Also returns A(p) = sum_i |c_i| G_i(p) over the
    in-support pairs, the scale against which rounding error is measured.
    """
    mu, _, _, c = split(params)
    P = precision(params)
    S = covariance(params)
    k2 = float(k) * float(k)
    V = np.zeros(grid.shape)
    A = np.zeros(grid.shape)
    lo = np.zeros(grid.shape)
    hi = np.zeros(grid.shape)
    namb = 0
    for i in range(mu.shape[0]):
        box = support_box(mu[i], S[i], k, grid)
        if box is None:
            continue
        dx, dy, dz = _box_offsets(box, mu[i], grid)
        m2 = _quad(P[i], dx, dy, dz)
        g = np.exp(-0.5 * m2)
        inside = m2 < k2
        sl = (slice(box[2][0], box[2][1] + 1), slice(box[1][0], box[1][1] + 1),
              slice(box[0][0], box[0][1] + 1))
        V[sl] += np.where(inside, c[i] * g, 0.0)
        A[sl] += np.where(inside, abs(c[i]) * g, 0.0)
        if band > 0.0:
            amb = np.abs(m2 - k2) < band
            namb += int(np.count_nonzero(amb))
            lo[sl] += np.where(inside & ~amb, c[i] * g, 0.0)
            hi[sl] += np.where(inside | amb, c[i] * g, 0.0)
    if band > 0.0:
        return V, A, (lo, hi, namb)
    return V, A


def count_pairs(params, grid: Grid, k):
    """Number of in-support (primitive, voxel) pairs, m^2 < k^2."""
    mu, _, _, _ = split(params)
    P = precision(params)
    S = covariance(params)
    tot = 0
    for i in range(mu.shape[0]):
        box = support_box(mu[i], S[i], k, grid)
        if box is None:
            continue
        dx, dy, dz = _box_offsets(box, mu[i], grid)
        tot += int(np.count_nonzero(_quad(P[i], dx, dy, dz) < float(k) * float(k)))
    return tot


# ----------------------------------------------------------------------------
# Loss and gradient
# ----------------------------------------------------------------------------

def loss(params, field, grid: Grid, k):
    V, _ = evaluate_windowed(params, grid, k)
    r = V - np.asarray(field, dtype=np.float64).reshape(grid.shape)
    return float(np.sum(r * r))


def loss_grad(params, field, grid: Grid, k, return_parts=False):
    """L = sum_p (V_k(p) - V(p))^2 and dL/dtheta as an (11, N) array.

    Per in-support pair, with r = 2 (V_k - V), e = r G and g = c e:
      dL/dc   = sum e
      dL/dmu  = P sum g d                       (dm^2/dmu = -2 P d)
      dL/dP   = -1/2 D,  D = sum g d d^T
      dL/dl_j = s_j^-2 (R^T D R)_jj             (dP/dl_j = -2 s_j^-2 r_j r_j^T)
      dL/dR   = -D R S^-2
      dL/dq_n = <dL/dR, dR/dq_n>  (R quadratic in the unit quaternion)
      dL/dq   = (I - q_n q_n^T) dL/dq_n / |q|
    """
    fld = np.asarray(field, dtype=np.float64).reshape(grid.shape)
    V, _ = evaluate_windowed(params, grid, k)
    res = V - fld
    L = float(np.sum(res * res))
    grad, parts = grad_from_residual(params, 2.0 * res, grid, k)
    if return_parts:
        return L, grad, parts
    return L, grad


def grad_from_residual(params, r, grid: Grid, k, window=True):
    """The gradient sums of ``loss_grad`` for a given residual r = dL/dV_k
    (for the squared error, 2 (V_k - V)) on every voxel: returns
    (dL/dtheta (11, N), the ten per-primitive sums (10, N)).  The primitives
    enter only through their own pairs, so a subset of the primitives gets
    exactly its part of the full gradient.  ``window=False`` visits every
    voxel of the grid for every primitive (brute force) instead of its
    support box; out-of-support pairs then add exact zeros."""
    mu, q, ell, c = split(params)
    qn, qnorm, qok = normalize_quat(q)
    R = rotation(qn)
    P = precision(params)
    S = covariance(params)
    k2 = float(k) * float(k)
    N = mu.shape[0]
    grad = np.zeros((NPARAM, N))
    parts = np.zeros((10, N))
    full = ((0, grid.nx - 1), (0, grid.ny - 1), (0, grid.nz - 1))
    for i in range(N):
        box = support_box(mu[i], S[i], k, grid) if window else full
        if box is None:
            continue
        dx, dy, dz = _box_offsets(box, mu[i], grid)
        m2 = _quad(P[i], dx, dy, dz)
        Gm = np.where(m2 < k2, np.exp(-0.5 * m2), 0.0)
        sl = (slice(box[2][0], box[2][1] + 1), slice(box[1][0], box[1][1] + 1),
              slice(box[0][0], box[0][1] + 1))
        e = r[sl] * Gm
        g = c[i] * e
        Se = np.sum(e)
        Sgd = np.array([np.sum(g * dx), np.sum(g * dy), np.sum(g * dz)])
        D = np.array([[np.sum(g * dx * dx), np.sum(g * dx * dy), np.sum(g * dx * dz)],
                      [np.sum(g * dy * dx), np.sum(g * dy * dy), np.sum(g * dy * dz)],
                      [np.sum(g * dz * dx), np.sum(g * dz * dy), np.sum(g * dz * dz)]])
        parts[:, i] = [Se, Sgd[0], Sgd[1], Sgd[2], D[0, 0], D[0, 1], D[0, 2],
                       D[1, 1], D[1, 2], D[2, 2]]
        si2 = np.exp(-2.0 * ell[i])
        grad[0:3, i] = P[i] @ Sgd
        RtDR = R[i].T @ D @ R[i]
        grad[7:10, i] = si2 * np.diag(RtDR)
        if qok[i]:
            dR = -D @ R[i] @ np.diag(si2)
            dRq = rotation_partials(qn[i])
            dqn = np.array([np.sum(dR * dRq[a]) for a in range(4)])
            proj = np.eye(4) - np.outer(qn[i], qn[i])
            grad[3:7, i] = proj @ dqn / qnorm[i]
        grad[10, i] = Se
    return grad, parts


def loss_grad_bruteforce(params, field, grid: Grid, k):
    """``loss_grad`` visiting every (primitive, voxel) pair of the grid: the
    field by ``evaluate_bruteforce``, the gradient by ``grad_from_residual``
    without support boxes."""
    fld = np.asarray(field, dtype=np.float64).reshape(grid.shape)
    res = evaluate_bruteforce(params, grid, k) - fld
    grad, _ = grad_from_residual(params, 2.0 * res, grid, k, window=False)
    return float(np.sum(res * res)), grad


def loss_grad_absolute(params, field, grid: Grid, k):
    """Sum over in-support pairs of |per-pair contribution| to dL/dtheta, (11, N).

    The same per-pair terms as ``loss_grad`` (r = 2 (V_k - V), g = c r G,
    d = p - mu), each taken in absolute value before summing: the scale
    against which float32 accumulation error in a gradient entry is measured
    (a gradient that is a small difference of large terms cannot be matched
    to 1e-3 of itself, only to 1e-3 of this).
    """
    mu, q, ell, c = split(params)
    qn, qnorm, qok = normalize_quat(q)
    R = rotation(qn)
    P = precision(params)
    S = covariance(params)
    k2 = float(k) * float(k)
    fld = np.asarray(field, dtype=np.float64).reshape(grid.shape)
    V, _ = evaluate_windowed(params, grid, k)
    r = 2.0 * (V - fld)
    N = mu.shape[0]
    out = np.zeros((NPARAM, N))
    for i in range(N):
        box = support_box(mu[i], S[i], k, grid)
        if box is None:
            continue
        dx, dy, dz = _box_offsets(box, mu[i], grid)
        m2 = _quad(P[i], dx, dy, dz)
        inside = m2 < k2
        if not np.any(inside):
            continue
        sl = (slice(box[2][0], box[2][1] + 1), slice(box[1][0], box[1][1] + 1),
              slice(box[0][0], box[0][1] + 1))
        G = np.exp(-0.5 * m2[inside])
        e = r[sl][inside] * G
        g = c[i] * e
        d = np.stack([dx[inside], dy[inside], dz[inside]], axis=1)      # [v, 3]
        out[10, i] = np.sum(np.abs(e))
        out[0:3, i] = np.sum(np.abs((g[:, None] * d) @ P[i].T), axis=0)
        si2 = np.exp(-2.0 * ell[i])
        proj = d @ R[i]                                                  # r_j^T d
        out[7:10, i] = si2 * np.sum(np.abs(g)[:, None] * proj * proj, axis=0)
        if qok[i]:
            Dp = g[:, None, None] * d[:, :, None] * d[:, None, :]        # [v, 3, 3]
            dR = -np.einsum("vij,jk->vik", Dp, R[i] @ np.diag(si2))
            dRq = rotation_partials(qn[i])
            dqn = np.einsum("vij,aij->va", dR, dRq)
            qg = dqn @ (np.eye(4) - np.outer(qn[i], qn[i])).T / qnorm[i]
            out[3:7, i] = np.sum(np.abs(qg), axis=0)
    return out


def _pair_jacobian(c, G, d, P, R, ell, qn, qnorm, qok):
    """d(c G(p))/dtheta for one primitive and one in-support voxel (11 values).

    The single-voxel case of the sums in ``loss_grad`` with r = 1: e = G,
    g = c G, D = g d d^T.
    """
    out = np.zeros(NPARAM)
    g = c * G
    out[0:3] = P @ (g * d)
    D = g * np.outer(d, d)
    si2 = np.exp(-2.0 * ell)
    out[7:10] = si2 * np.diag(R.T @ D @ R)
    if qok:
        dR = -D @ R @ np.diag(si2)
        dRq = rotation_partials(qn)
        dqn = np.array([np.sum(dR * dRq[a]) for a in range(4)])
        out[3:7] = (np.eye(4) - np.outer(qn, qn)) @ dqn / qnorm
    out[10] = G
    return out


def boundary_slack(params, field, grid: Grid, k, band):
    """How far dL/dtheta can move when pairs near the cut change sides.

    A pair whose float64 m^2 lies within ``band`` of k^2 may be decided either
    way by a float32 evaluator.  Flipping pair (i, p) (first order):
      * adds or drops the direct term r(p) d(c_i G_i(p))/dtheta_i;
      * moves Vhat(p) by c_i G_i(p), so r(p) by 2 c_i G_i(p), which changes
        dL/dtheta_j by 2 c_i G_i(p) d(c_j G_j(p))/dtheta_j for every j whose
        support holds p (i included).
    Returns the (11, N) sum of the magnitudes of both over every such pair (a
    bound for any set of flips) and the number of pairs.
    """
    mu, q, ell, c = split(params)
    qn, qnorm, qok = normalize_quat(q)
    R = rotation(qn)
    P = precision(params)
    S = covariance(params)
    k2 = float(k) * float(k)
    fld = np.asarray(field, dtype=np.float64).reshape(grid.shape)
    V, _ = evaluate_windowed(params, grid, k)
    r = 2.0 * (V - fld)
    N = mu.shape[0]
    slack = np.zeros((NPARAM, N))
    amb = []
    for i in range(N):
        box = support_box(mu[i], S[i], math.sqrt(k2 + band), grid)  # pairs just outside too
        if box is None:
            continue
        dx, dy, dz = _box_offsets(box, mu[i], grid)
        m2 = _quad(P[i], dx, dy, dz)
        hit = np.abs(m2 - k2) < band
        for kk, jj, ii in zip(*np.nonzero(hit)):
            amb.append((i, box[0][0] + ii, box[1][0] + jj, box[2][0] + kk))
    for i, ix, iy, iz in amb:
        p = np.array([grid.x0 + ix, grid.y0 + iy, grid.z0 + iz], dtype=np.float64)
        d = p - mu[i]
        Gi = math.exp(-0.5 * float(d @ P[i] @ d))
        Ji = _pair_jacobian(c[i], Gi, d, P[i], R[i], ell[i], qn[i], qnorm[i], qok[i])
        slack[:, i] += abs(r[iz, iy, ix]) * np.abs(Ji)
        shift = 2.0 * abs(c[i]) * Gi
        D = p[None, :] - mu
        m2all = np.einsum("nj,njk,nk->n", D, P, D)
        for j in np.nonzero(m2all < k2 + band)[0]:
            Gj = math.exp(-0.5 * float(m2all[j]))
            Jj = _pair_jacobian(c[j], Gj, D[j], P[j], R[j], ell[j], qn[j], qnorm[j], qok[j])
            slack[:, j] += shift * np.abs(Jj)
    return slack, len(amb)


# ----------------------------------------------------------------------------
# Adam and refinement
# ----------------------------------------------------------------------------

@dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    t: int = 0

    @staticmethod
    def zeros(n):
        return AdamState(np.zeros((NPARAM, n)), np.zeros((NPARAM, n)), 0)


def adam_update(params, grad, state: AdamState, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                ell_clamp=None):
    """One bias-corrected Adam step on every parameter (Kingma and Ba).

    ``ell_clamp`` = (lo, hi) optionally clamps the log-scales after the step.
    Returns (new_params, number of clamped log-scale entries).
    """
    p = np.asarray(params, dtype=np.float64).copy()
    g = np.asarray(grad, dtype=np.float64)
    state.t += 1
    state.m = beta1 * state.m + (1.0 - beta1) * g
    state.v = beta2 * state.v + (1.0 - beta2) * g * g
    mhat = state.m / (1.0 - beta1 ** state.t)
    vhat = state.v / (1.0 - beta2 ** state.t)
    p -= lr * mhat / (np.sqrt(vhat) + eps)
    nclamp = 0
    if ell_clamp is not None:
        lo, hi = ell_clamp
        ell = p[7:10]
        nclamp = int(np.count_nonzero((ell < lo) | (ell > hi)))
        p[7:10] = np.clip(ell, lo, hi)
    return p, nclamp


def refine(params, field, grid: Grid, k, iters, lr, beta1=0.9, beta2=0.999, eps=1e-8,
           state: AdamState | None = None, ell_clamp=None):
    """``iters`` rounds of (evaluate, loss, gradient, Adam).

    Returns (params, state, losses) where losses[t] is L before update t.
    """
    p = np.asarray(params, dtype=np.float64).copy()
    if state is None:
        state = AdamState.zeros(p.shape[1])
    losses = []
    for _ in range(iters):
        L, g = loss_grad(p, field, grid, k)
        losses.append(L)
        p, _ = adam_update(p, g, state, lr, beta1, beta2, eps, ell_clamp)
    return p, state, np.array(losses)


def psnr_from_mse(mse):
    """PSNR on a field normalised to [0, 1] (Sec. IV-C): 10 log10(1 / MSE)."""
    return 10.0 * math.log10(1.0 / mse)


def sampled_mse(pred, field, n, seed):
    """MSE at ``n`` voxel centres drawn uniformly with replacement (Sec. IV-C)."""
    a = np.asarray(pred, dtype=np.float64).ravel()
    b = np.asarray(field, dtype=np.float64).ravel()
    idx = np.random.default_rng(seed).integers(0, a.size, size=n)
    d = a[idx] - b[idx]
    return float(np.mean(d * d))


def encoded_bytes(n, header_bytes):
    """Full-precision encoded size, Sec. III-J eq:size: 48 N + H."""
    return 48 * int(n) + int(header_bytes)


def compression_ratio(n_voxels, bytes_per_voxel, n, header_bytes):
    """Sec. III-J eq:cr: S_src / S_enc(N)."""
    return n_voxels * bytes_per_voxel / encoded_bytes(n, header_bytes)
