"""Oracle: structure-aware fixed-budget allocation (paper Sec. III-E; Table
"Implemented pipeline stages", rows S1a-S1e).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  NumPy, float64 except
where a float32 value decides a discrete choice (then the same float32 value
that the device computes is used, see below).

Steps, in the paper's order.  The constants the paper does not print are
readings of it, stated where they are used: the counter-based random numbers,
the 4096-seed subsample, the 7^3 tensor box, the 99th-percentile gradient
scale, the elongation rule and its cap, and the scale floor:

S1a  gradient magnitude: central differences (one-sided at the grid faces) of
     the float32 field; g = |grad V| formed in float64 from the float32
     differences and rounded to float32 (``g32``), so that the device, which
     does the same, reaches the same value bit for bit.
S1b  budget draw: N_det = floor(0.55 N + 1/2) detail seeds drawn without
     replacement with probability proportional to g over the occupied domain
     O = {V > 0.02} (eligible: g > 0), and N_cov = N - N_det coverage seeds
     drawn uniformly over O; distinct positions within each draw.  A request
     with N_det > |E| or N_cov > |O| is infeasible (Sec. V-B) and reports the
     shortfall.  Weighted sampling without replacement uses exponential clocks
     (Efraimidis-Spirakis): key_v = -ln(u_v) / g_v, the N_det smallest keys,
     ties to the lower voxel index; u_v from the SplitMix64 finaliser of a
     counter (seed, stream, v).  Off-grid jitter mu = c + u - 1/2 per axis.
S1c  group scale: the lower median, over a strided subsample of at most 4096
     seeds of the group, of the distance to the nearest other seed of the
     group.
S1d  per-seed structure tensor J = sum over the 7^3 box (clipped) of
     grad V grad V^T; eigenvalues l1 >= l2 >= l3; tangent = e3 (smallest).
S1e  R = [e3, e2, e1] (right-handed), scales (s_t, s_b, s_b) with
     s_t = min(s_b (1 + 2 gh), 3 s_b), gh = clip(g(c) / g99, 0, 1), g99 the
     99th-percentile order statistic of g32 over O; every scale clipped to
     [0.25, max(dims) / 16]; values a_i = V(c_i) and a global weight
     kappa = <U, V> / <U, U> with U = sum_i a_i G_i, c_i = kappa a_i.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

from . import field as F

OCC_THRESHOLD = 0.02
DETAIL_FRACTION = 0.55
SUBSAMPLE = 4096
ST_RADIUS = 3            # 7^3 box
MIN_SCALE = 0.25
CAP_DIVISOR = 16.0
MAX_ELONGATION = 3.0

STREAM_DETAIL, STREAM_COVER = 1, 2
STREAM_JITTER = 3        # + 3 * group + axis

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_STREAM_MUL = 0xD1B54A32D192ED03


class BudgetInfeasible(Exception):
    def __init__(self, shortfall, n_det, n_cov, n_eligible, n_occupied):
        super().__init__(f"budget infeasible: shortfall {shortfall}")
        self.shortfall = shortfall
        self.n_det, self.n_cov = n_det, n_cov
        self.n_eligible, self.n_occupied = n_eligible, n_occupied


# ----------------------------------------------------------------------------- RNG

def splitmix64(x):
    """SplitMix64 output function (Steele, Lea and Flood 2014) of uint64 x."""
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(_GOLDEN))
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def hash_bits(seed, stream, idx):
    """64 random bits for counter (seed, stream, idx)."""
    with np.errstate(over="ignore"):
        base = splitmix64(np.uint64(seed & _M64) ^ (np.uint64(stream) * np.uint64(_STREAM_MUL)))
        return splitmix64(base ^ np.asarray(idx, dtype=np.uint64))


def uniform01(seed, stream, idx):
    """Uniform in (0, 1]: (top 53 bits + 1) * 2^-53, exact in float64."""
    b = (hash_bits(seed, stream, idx) >> np.uint64(11)) + np.uint64(1)
    return b.astype(np.float64) * (2.0 ** -53)


# ----------------------------------------------------------------------------- S1a

def gradient_parts(field):
    """float32 half-differences (central) / differences (one-sided at faces).

    Returns (gx, gy, gz) float32 arrays shaped like ``field`` ([z, y, x])."""
    v = np.asarray(field, dtype=np.float32)
    out = []
    for axis in (2, 1, 0):              # x, y, z
        d = np.empty_like(v)
        n = v.shape[axis]
        sl = lambda a, b: tuple(slice(a, b) if ax == axis else slice(None) for ax in range(3))
        if n == 1:
            d[...] = 0.0
        else:
            d[sl(1, n - 1)] = np.float32(0.5) * (v[sl(2, n)] - v[sl(0, n - 2)])
            d[sl(0, 1)] = v[sl(1, 2)] - v[sl(0, 1)]
            d[sl(n - 1, n)] = v[sl(n - 1, n)] - v[sl(n - 2, n - 1)]
        out.append(d)
    return tuple(out)


def gradient_magnitude32(field):
    gx, gy, gz = gradient_parts(field)
    x, y, z = gx.astype(np.float64), gy.astype(np.float64), gz.astype(np.float64)
    return np.sqrt((x * x + y * y) + z * z).astype(np.float32)


# ----------------------------------------------------------------------------- S1b

def split_budget(n):
    n_det = int(math.floor(DETAIL_FRACTION * n + 0.5))
    return n_det, n - n_det


def max_feasible_budget(n_eligible, n_occupied):
    """Largest N with N_det <= |E| and N_cov <= |O| (Sec. V-B arithmetic)."""
    lo, hi = 0, 4 * (n_occupied + n_eligible) + 4
    while lo < hi:
        mid = (lo + hi + 1) // 2
        d, c = split_budget(mid)
        if d <= n_eligible and c <= n_occupied:
            lo = mid
        else:
            hi = mid - 1
    return lo


def smallest_k(keys, cand_idx, k):
    """Indices (from cand_idx) of the k smallest keys, ties to lower index,
    returned in increasing voxel index."""
    order = np.lexsort((cand_idx, keys))
    return np.sort(cand_idx[order[:k]])


def draw_seeds(field, g32, n, seed):
    v = np.asarray(field, dtype=np.float32).ravel()
    g = np.asarray(g32, dtype=np.float32).ravel()
    occ = np.flatnonzero(v > np.float32(OCC_THRESHOLD))
    elig = occ[g[occ] > 0]
    n_det, n_cov = split_budget(n)
    short = max(n_det - elig.size, n_cov - occ.size, 0)
    if short > 0:
        raise BudgetInfeasible(short, n_det, n_cov, elig.size, occ.size)
    u = uniform01(seed, STREAM_DETAIL, elig)
    kd = -np.log(u) / g[elig].astype(np.float64)
    det = smallest_k(kd, elig, n_det)
    kc = hash_bits(seed, STREAM_COVER, occ) >> np.uint64(11)
    cov = smallest_k(kc, occ, n_cov)
    return det, cov, elig.size, occ.size


def jitter_centers(vox, shape, origin, seed, group):
    nz, ny, nx = shape
    i = vox % nx
    j = (vox // nx) % ny
    k = vox // (nx * ny)
    base = (i + origin[0], j + origin[1], k + origin[2])
    mu = np.empty((3, vox.size))
    for a in range(3):
        u = uniform01(seed, STREAM_JITTER + 3 * group + a, vox)
        mu[a] = (base[a] + u) - 0.5
    return mu.astype(np.float32)


# ----------------------------------------------------------------------------- S1c

def group_spacing(mu32):
    """Lower median of nearest-neighbour distances over a strided subsample."""
    mu = np.asarray(mu32, dtype=np.float32).astype(np.float64)
    n = mu.shape[1]
    if n < 2:
        return 1.0
    stride = -(-n // SUBSAMPLE)
    sub = np.arange(0, n, stride)
    best = np.full(sub.size, np.inf)
    for a in range(0, sub.size, 256):
        s = sub[a:a + 256]
        dx = mu[0][None, :] - mu[0][s][:, None]
        dy = mu[1][None, :] - mu[1][s][:, None]
        dz = mu[2][None, :] - mu[2][s][:, None]
        d2 = (dx * dx + dy * dy) + dz * dz
        d2[np.arange(s.size), s] = np.inf
        best[a:a + 256] = d2.min(axis=1)
    best.sort()
    return math.sqrt(best[(best.size - 1) // 2])


# ----------------------------------------------------------------------------- S1d

def structure_tensor(parts, vox_ijk, radius=ST_RADIUS):
    nz, ny, nx = parts[0].shape
    i, j, k = vox_ijk
    sl = (slice(max(k - radius, 0), min(k + radius + 1, nz)),
          slice(max(j - radius, 0), min(j + radius + 1, ny)),
          slice(max(i - radius, 0), min(i + radius + 1, nx)))
    a, b, c = (p[sl].astype(np.float64).ravel() for p in parts)
    return np.array([[a @ a, a @ b, a @ c], [a @ b, b @ b, b @ c], [a @ c, b @ c, c @ c]])


def frame_from_tensor(J):
    """R = [e3, e2, e1] with l1 >= l2 >= l3, each eigenvector's largest-magnitude
    component positive, then the third column flipped if needed for det R = +1.
    Also returns the eigenvalues (l1, l2, l3)."""
    if np.trace(J) < 1e-12:
        return np.eye(3), np.zeros(3)
    w, v = np.linalg.eigh(J)            # ascending
    lam = w[::-1]
    e1, e2, e3 = v[:, 2], v[:, 1], v[:, 0]
    cols = []
    for e in (e3, e2, e1):
        if e[np.argmax(np.abs(e))] < 0:
            e = -e
        cols.append(e)
    R = np.stack(cols, axis=1)
    if np.linalg.det(R) < 0:
        R[:, 2] = -R[:, 2]
    return R, lam


def quat_from_rotation(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix, w >= 0."""
    t = np.trace(R)
    if t > 0:
        s = math.sqrt(t + 1.0) * 2
        q = np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s,
                      (R[1, 0] - R[0, 1]) / s])
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = np.array([(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s,
                      (R[0, 2] + R[2, 0]) / s])
    elif R[1, 1] > R[2, 2]:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = np.array([(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s,
                      (R[1, 2] + R[2, 1]) / s])
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = np.array([(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s,
                      (R[1, 2] + R[2, 1]) / s, 0.25 * s])
    q /= np.linalg.norm(q)
    return -q if q[0] < 0 else q


# ----------------------------------------------------------------------------- S1e

def percentile_order_stat(values32, q=0.99):
    s = np.sort(np.asarray(values32, dtype=np.float32).ravel())
    return s[int(math.floor(q * (s.size - 1)))]


def lsq_weight(U, V):
    U = np.asarray(U, dtype=np.float64).ravel()
    V = np.asarray(V, dtype=np.float64).ravel()
    uu = float(U @ U)
    return float(U @ V) / uu if uu > 0 else 0.0


def frame_and_scales(parts, gflat, vi, grid: F.Grid, s_base, g99, s_cap):
    """Orientation and log-scales of the primitive seeded at voxel vi (S1d):
    the frame of the structure tensor of the 7^3 box around the seed, the
    tangent axis stretched by 1 + 2 |grad V| / g99 (at most 3x), every scale
    within [0.25, s_cap].  Returns (quaternion, log-scales, eigenvalues)."""
    i = int(vi % grid.nx)
    j = int((vi // grid.nx) % grid.ny)
    kk = int(vi // (grid.nx * grid.ny))
    J = structure_tensor(parts, (i, j, kk))
    R, lam = frame_from_tensor(J)
    gh = min(max(float(gflat[vi]) / g99, 0.0), 1.0) if g99 > 0 else 0.0
    st = min(s_base * (1.0 + 2.0 * gh), MAX_ELONGATION * s_base)
    s = np.clip(np.array([st, s_base, s_base]), MIN_SCALE, max(s_cap, MIN_SCALE))
    return quat_from_rotation(R), np.log(s), lam


@dataclass
class AllocInfo:
    n_det: int
    n_cov: int
    n_eligible: int
    n_occupied: int
    det_voxels: np.ndarray
    cov_voxels: np.ndarray
    s_base: tuple
    g99: float
    kappa: float
    eigvals: np.ndarray = dc_field(default=None)


def allocate(field, grid: F.Grid, n, seed, k=3.0):
    """The full S1a-S1e allocation; returns (params float64 (11, n), AllocInfo).

    Primitives are ordered detail seeds first, then coverage seeds, each in
    increasing voxel index."""
    v = np.asarray(field, dtype=np.float32).reshape(grid.shape)
    parts = gradient_parts(v)
    g32 = gradient_magnitude32(v)
    det, cov, n_el, n_oc = draw_seeds(v, g32, n, seed)
    origin = (grid.x0, grid.y0, grid.z0)
    mus = [jitter_centers(det, grid.shape, origin, seed, 0),
           jitter_centers(cov, grid.shape, origin, seed, 1)]
    s_base = (group_spacing(mus[0]), group_spacing(mus[1]))
    occ = v.ravel() > np.float32(OCC_THRESHOLD)
    g99 = float(percentile_order_stat(g32.ravel()[occ]))
    s_cap = max(grid.nx, grid.ny, grid.nz) / CAP_DIVISOR
    params = np.zeros((11, n))
    eig = np.zeros((n, 3))
    col = 0
    gflat = g32.ravel()
    for group, vox in enumerate((det, cov)):
        sb = s_base[group]
        for t, vi in enumerate(vox):
            q, ell, lam = frame_and_scales(parts, gflat, int(vi), grid, sb, g99, s_cap)
            params[0:3, col] = mus[group][:, t]
            params[3:7, col] = q
            params[7:10, col] = ell
            params[10, col] = float(v.ravel()[vi])
            eig[col] = lam
            col += 1
    U, _ = F.evaluate_windowed(params, grid, k)
    kappa = lsq_weight(U, v)
    params[10] *= kappa
    info = AllocInfo(len(det), len(cov), n_el, n_oc, det, cov, s_base, g99, kappa, eig)
    return params, info
