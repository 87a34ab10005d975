"""Oracle: the warm-start network and its features and targets.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  NumPy float64.

The paper does not describe a learned component; the network is defined by
its shapes only (16 -> 128 -> 128 -> 11 with GELU, BF16 operands, FP32
accumulation, trained on pairs of (allocated primitive -> refined primitive)
produced by the encoder itself).  The readings used here:

* Features (16 per primitive, at allocation): the structure-tensor
  eigenvalues at the seed voxel as log1p(lambda / g99^2) (3), its eigenvectors
  e1, e2, e3 (9, each with its largest-magnitude component positive), the
  gradient magnitude at the seed over g99 (1), mean and variance of V over the
  primitive's k-sigma box (2), and the group flag (1 = detail seed).
* Targets (11): theta_refined - theta_alloc, with the refined quaternion
  normalised and sign-aligned to the allocated one.
* Network: y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 on standardised x and
  standardised targets; GELU(z) = z/2 (1 + erf(z / sqrt 2)).
* Loss: mean over the batch and the 11 outputs of the squared error.
* ``bf16=True`` rounds every GEMM operand to bfloat16 (round to nearest even)
  before the product, with float64 accumulation: the device's arithmetic up to
  its float32 accumulation order.
"""
from __future__ import annotations

import math

import numpy as np

from . import alloc as A
from . import field as F

D_IN, D_H, D_OUT = 16, 128, 11


def bf16_round(x):
    """Round float64/float32 values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    nan = np.isnan(f)
    out = (r << np.uint64(16)).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def _mm(a, b, bf16):
    if bf16:
        return bf16_round(a) @ bf16_round(b)
    return a @ b


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases; float64."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, (o, i) in (("1", (D_H, D_IN)), ("2", (D_H, D_H)), ("3", (D_OUT, D_H))):
        b = math.sqrt(6.0 / i)
        p["W" + name] = rng.uniform(-b, b, size=(o, i))
        p["b" + name] = np.zeros(o)
    return p


def forward(p, X, bf16=False):
    """X [B, 16] (standardised) -> (Y [B, 11], cache for backward)."""
    Z1 = _mm(X, p["W1"].T, bf16) + p["b1"]
    H1 = gelu(Z1)
    Z2 = _mm(H1, p["W2"].T, bf16) + p["b2"]
    H2 = gelu(Z2)
    Y = _mm(H2, p["W3"].T, bf16) + p["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grads(p, X, T, bf16=False):
    """Mean squared error over batch and outputs, and its gradients."""
    Y, (X, Z1, H1, Z2, H2) = forward(p, X, bf16)
    B = X.shape[0]
    R = Y - T
    L = float(np.mean(R * R))
    dY = 2.0 * R / (B * D_OUT)
    g = {}
    g["W3"] = _mm(dY.T, H2, bf16)
    g["b3"] = dY.sum(axis=0)
    dH2 = _mm(dY, p["W3"], bf16)
    dZ2 = dH2 * gelu_grad(Z2)
    g["W2"] = _mm(dZ2.T, H1, bf16)
    g["b2"] = dZ2.sum(axis=0)
    dH1 = _mm(dZ2, p["W2"], bf16)
    dZ1 = dH1 * gelu_grad(Z1)
    g["W1"] = _mm(dZ1.T, X, bf16)
    g["b1"] = dZ1.sum(axis=0)
    return L, g


def adam(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Bias-corrected Adam on every tensor of the network; state = {'t', 'm', 'v'}."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k in p:
        m = state.setdefault("m", {}).get(k, np.zeros_like(p[k]))
        v = state.setdefault("v", {}).get(k, np.zeros_like(p[k]))
        m = beta1 * m + (1 - beta1) * g[k]
        v = beta2 * v + (1 - beta2) * g[k] * g[k]
        state["m"][k], state["v"][k] = m, v
        out[k] = p[k] - lr * (m / (1 - beta1 ** t)) / (np.sqrt(v / (1 - beta2 ** t)) + eps)
    return out


# ----------------------------------------------------------------------------- features

def box_stats(field, grid: F.Grid, params, k):
    """Mean and (population) variance of V over each primitive's k-sigma box."""
    v = np.asarray(field, dtype=np.float64).reshape(grid.shape)
    mu, _, _, _ = F.split(params)
    S = F.covariance(params)
    out = np.zeros((params.shape[1], 2))
    for i in range(params.shape[1]):
        box = F.support_box(mu[i], S[i], k, grid)
        if box is None:
            continue
        (ia, ib), (ja, jb), (ka, kb) = box
        blk = v[ka:kb + 1, ja:jb + 1, ia:ib + 1]
        out[i] = (blk.mean(), blk.var())
    return out


def features(field, grid: F.Grid, params, n_detail, g99, k):
    """The 16 features of every allocated primitive (seed voxel = round(mu))."""
    v = np.asarray(field, dtype=np.float32).reshape(grid.shape)
    parts = A.gradient_parts(v)
    g32 = A.gradient_magnitude32(v).ravel()
    mu = np.asarray(params[0:3], dtype=np.float64)
    n = params.shape[1]
    X = np.zeros((n, D_IN))
    bs = box_stats(v, grid, params, k)
    for i in range(n):
        ii = int(np.floor(mu[0, i] - grid.x0 + 0.5))
        jj = int(np.floor(mu[1, i] - grid.y0 + 0.5))
        kk = int(np.floor(mu[2, i] - grid.z0 + 0.5))
        ii = min(max(ii, 0), grid.nx - 1)
        jj = min(max(jj, 0), grid.ny - 1)
        kk = min(max(kk, 0), grid.nz - 1)
        J = A.structure_tensor(parts, (ii, jj, kk))
        R, lam = A.frame_from_tensor(J)
        e3, e2, e1 = R[:, 0], R[:, 1], R[:, 2]
        # the frame's third column may have been flipped for handedness; the
        # feature uses the canonical sign (largest-magnitude component > 0)
        if e1[np.argmax(np.abs(e1))] < 0:
            e1 = -e1
        gg = g99 * g99 if g99 > 0 else 1.0
        X[i, 0:3] = np.log1p(np.maximum(lam, 0.0) / gg)
        X[i, 3:6], X[i, 6:9], X[i, 9:12] = e1, e2, e3
        vox = ii + grid.nx * (jj + grid.ny * kk)
        X[i, 12] = float(g32[vox]) / g99 if g99 > 0 else 0.0
        X[i, 13:15] = bs[i]
        X[i, 15] = 1.0 if i < n_detail else 0.0
    return X


def targets(theta_alloc, theta_ref):
    """theta_ref - theta_alloc per primitive, [n, 11], refined q sign-aligned."""
    a = np.asarray(theta_alloc, dtype=np.float64)
    r = np.asarray(theta_ref, dtype=np.float64).copy()
    qn = r[3:7] / np.maximum(np.linalg.norm(r[3:7], axis=0), 1e-30)
    flip = np.sum(qn * a[3:7], axis=0) < 0
    qn[:, flip] *= -1
    r[3:7] = qn
    return (r - a).T


# ----------------------------------------------------------------------------- training loop

def column_stats(X):
    """Per-column mean and population standard deviation of a [rows, cols]
    matrix, the standardisation the network is trained with.  A column whose
    deviation is at most 1e-6 keeps a scale of 1 (it carries no information)."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    sd = np.sqrt(np.maximum((X * X).mean(axis=0) - mean * mean, 0.0))
    return mean, np.where(sd > 1e-6, sd, 1.0)


def epoch_permutation(n, seed, epoch):
    """Order in which epoch `epoch` visits the n training rows: the rows sorted
    by a 32-bit key drawn from the counter generator of ``oracle.alloc``
    (SplitMix64 of (seed, stream = epoch, row), top 32 bits), ties kept in row
    order.  Random numbers the training draws are thus a function of the seed
    alone, written here from the generator's published definition."""
    keys = (A.hash_bits(seed, epoch, np.arange(n, dtype=np.uint64)) >> np.uint64(32))
    return np.argsort(keys.astype(np.uint64), kind="stable")


def flat_to_params(flat):
    """The library's flat layout (W1, b1, W2, b2, W3, b3) as a dict of float64."""
    flat = np.asarray(flat, dtype=np.float64)
    p, off = {}, 0
    for name, shape in (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
                        ("W3", (D_OUT, D_H)), ("b3", (D_OUT,))):
        size = int(np.prod(shape))
        p[name] = flat[off:off + size].reshape(shape).copy()
        off += size
    return p


def train(p, X, T, epochs, batch, lr, seed, bf16=True, stats_dtype=np.float32):
    """Mini-batch training of the network on raw features X [n, 16] and raw
    targets T [n, 11]: standardise both with their column statistics (held in
    ``stats_dtype``, the precision the statistics are stored in beside the
    weights), then for every epoch visit the rows in ``epoch_permutation``
    order in batches of `batch` rows (the last one may be short) and take one
    Adam step (``adam``) on each batch's mean squared error.

    Returns (weights, stats, per-epoch mean batch loss); stats =
    (feature mean, feature std, target mean, target std)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    fm, fs = (a.astype(stats_dtype).astype(np.float64) for a in column_stats(X))
    tm, ts = (a.astype(stats_dtype).astype(np.float64) for a in column_stats(T))
    Xs = (X - fm) / fs
    Ts = (T - tm) / ts
    n = X.shape[0]
    state = {}
    hist = []
    nb = (n + batch - 1) // batch
    for ep in range(epochs):
        perm = epoch_permutation(n, seed, ep)
        tot = 0.0
        for b in range(nb):
            rows = perm[b * batch:(b + 1) * batch]
            L, g = loss_and_grads(p, Xs[rows], Ts[rows], bf16=bf16)
            tot += L
            p = adam(p, g, state, lr)
        hist.append(tot / nb)
    return p, (fm, fs, tm, ts), np.array(hist)


# ----------------------------------------------------------------------------- warm start

def destandardise(Y, tmean, tstd):
    """Network outputs on the standardised scale [n, 11] -> parameter
    corrections Delta [n, 11] in the units of the 11 parameters."""
    return np.asarray(Y, dtype=np.float64) * np.asarray(tstd, dtype=np.float64) \
        + np.asarray(tmean, dtype=np.float64)


WARM_ALPHAS = (1.0, 0.5, 0.25)


def warmstart(theta_alloc, Y, tmean, tstd, loss_fn, alphas=WARM_ALPHAS):
    """Apply the network's correction to an allocation, with plain refinement's
    starting point as the fallback: theta = theta_alloc + alpha * Delta for
    alpha = 1, 1/2, 1/4 in turn, keeping the first whose loss (``loss_fn``,
    the full-grid sum of squares) is below the allocation's; if none is, the
    allocation is kept unchanged.

    theta_alloc [11, n]; Y [n, 11] standardised outputs.  Returns
    (applied, losses, theta): applied = 0 (fallback) or the 1-based index of
    the alpha kept; losses [4] = the allocation's loss and the loss at each
    alpha tried (NaN where not tried)."""
    theta_alloc = np.asarray(theta_alloc, dtype=np.float64)
    delta = destandardise(Y, tmean, tstd).T
    losses = [float(loss_fn(theta_alloc)), math.nan, math.nan, math.nan]
    for j, alpha in enumerate(alphas):
        theta = theta_alloc + alpha * delta
        losses[j + 1] = float(loss_fn(theta))
        if math.isfinite(losses[j + 1]) and losses[j + 1] < losses[0]:
            return j + 1, np.array(losses), theta
    return 0, np.array(losses), theta_alloc.copy()
