"""Seeded synthetic target fields and primitive sets.

These stand in for the paper's datasets (Sec. IV-A), which are not available:

* ``mixture_field``  -- a signed sum of random anisotropic Gaussians plus white
  noise (the small "plain method, tiny" workload: 64^3, 200 Gaussians with
  scales 1-4 voxels and weights U[-1, 1], noise 0.01).
* ``spectral_field`` -- a Gaussian random field whose shell energy spectrum
  falls as k^-5/3 (Kolmogorov-like; per-mode amplitude |k|^-11/6), min-max
  normalised to [0, 1] (the "mid" workload, 256^3).
* ``fronts_field``   -- tanh level-set fronts of noisy spheres plus a 0.1
  amplitude spectral background, normalised to [0, 1]; a combustion-like field
  at paper scale (1024^3, the grid size of the paper's largest volumes).

All draws are seeded.  ``mixture_field`` is NumPy float64; the spectral
generators run in torch on any device so that paper-scale fields can be drawn
directly in device memory.  Arrays are indexed [z, y, x] (x fastest).
"""
from __future__ import annotations


import numpy as np

PARAM_NAMES = ("mu_x", "mu_y", "mu_z", "q_w", "q_x", "q_y", "q_z",
               "l_x", "l_y", "l_z", "c")


def random_params(n, extent, seed, scale_range=(1.0, 4.0), weight_range=(-1.0, 1.0),
                  unit_quat=True, margin=0.0):
    """Random primitive set, float64 array (11, n) in PARAM_NAMES order.

    Centres uniform in [margin, extent - 1 - margin]^3 (extent may be a 3-tuple
    (nx, ny, nz)), orientation a uniformly random rotation (normalised N(0,1)^4
    quaternion; left un-normalised when ``unit_quat`` is False), scales uniform
    in ``scale_range`` voxels, weights uniform in ``weight_range``.
    """
    rng = np.random.default_rng(seed)
    ext = np.broadcast_to(np.asarray(extent, dtype=np.float64), (3,))
    p = np.empty((11, n))
    for j in range(3):
        p[j] = rng.uniform(margin, ext[j] - 1 - margin, size=n)
    q = rng.standard_normal((n, 4))
    if unit_quat:
        q /= np.linalg.norm(q, axis=1, keepdims=True)
    else:
        q *= rng.uniform(0.5, 2.0, size=(n, 1)) / np.linalg.norm(q, axis=1, keepdims=True)
    p[3:7] = q.T
    p[7:10] = np.log(rng.uniform(scale_range[0], scale_range[1], size=(3, n)))
    p[10] = rng.uniform(weight_range[0], weight_range[1], size=n)
    return p


def _rot_from_quat(q):
    # Rotation of a unit quaternion written as (w^2 - v.v) I + 2 v v^T + 2 w [v]x.
    w = q[0]
    v = q[1:4]
    vx = np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])
    return (w * w - v @ v) * np.eye(3) + 2.0 * np.outer(v, v) + 2.0 * w * vx


def mixture_field(params, shape, noise=0.0, seed=0):
    """Untruncated sum of the given Gaussians on an [nz, ny, nx] grid, float64.

    Each term is c exp(-|S^-1 R^T (p - mu)|^2 / 2); optional white noise of
    standard deviation ``noise`` (seeded) is added.
    """
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    out = np.zeros(pts.shape[0])
    p = np.asarray(params, dtype=np.float64)
    for i in range(p.shape[1]):
        q = p[3:7, i] / np.linalg.norm(p[3:7, i])
        R = _rot_from_quat(q)
        s = np.exp(p[7:10, i])
        z = ((pts - p[0:3, i]) @ R) / s
        out += p[10, i] * np.exp(-0.5 * np.sum(z * z, axis=1))
    out = out.reshape(shape)
    if noise > 0:
        out = out + np.random.default_rng(seed + 7919).normal(0.0, noise, size=shape)
    return out


def tiny_mixture(seed=0, n=64, count=200, noise=0.01, normalize=False):
    """The 64^3 signed-mixture workload: (field float32 [n,n,n], generating params)."""
    params = random_params(count, n, seed)
    f = mixture_field(params, (n, n, n), noise=noise, seed=seed)
    if normalize:
        f = (f - f.min()) / (f.max() - f.min())
    return f.astype(np.float32), params


def minmax01(t):
    lo = t.min()
    hi = t.max()
    return (t - lo) / (hi - lo)


def spectral_field(shape, seed, device="cpu", amp_exponent=-11.0 / 6.0, normalize="minmax"):
    """Gaussian random field with per-mode amplitude |k|^amp_exponent (DC removed).

    The default exponent gives a shell energy spectrum ~ k^-5/3.  ``normalize``:
    "minmax" -> [0, 1]; "std" -> zero mean, unit standard deviation; None -> raw.
    Returns a float32 torch tensor of ``shape`` = (nz, ny, nx) on ``device``.
    """
    import torch

    nz, ny, nx = shape
    gen = torch.Generator(device=device).manual_seed(int(seed))
    x = torch.randn((nz, ny, nx), generator=gen, device=device, dtype=torch.float32)
    spec = torch.fft.rfftn(x)
    del x
    kx = torch.arange(nx // 2 + 1, device=device, dtype=torch.float32)
    ky = torch.fft.fftfreq(ny, d=1.0 / ny, device=device).to(torch.float32)
    kz = torch.fft.fftfreq(nz, d=1.0 / nz, device=device).to(torch.float32)
    kxy2 = ky[:, None] ** 2 + kx[None, :] ** 2
    chunk = max(1, (1 << 26) // max(1, kxy2.numel()))
    for z0 in range(0, nz, chunk):
        kk = torch.sqrt(kz[z0:z0 + chunk, None, None] ** 2 + kxy2[None])
        amp = torch.where(kk > 0, kk.clamp_min(1e-30) ** amp_exponent, torch.zeros_like(kk))
        spec[z0:z0 + chunk] *= amp
        del kk, amp
    f = torch.fft.irfftn(spec, s=(nz, ny, nx))
    del spec
    if normalize == "minmax":
        f = minmax01(f)
    elif normalize == "std":
        f = (f - f.mean()) / f.std()
    return f.contiguous()


def fronts_field(n, seed, device="cpu", n_spheres=32, radius_range=(48.0, 192.0),
                 width_range=(2.0, 8.0), radius_jitter=0.1, background=0.1):
    """Combustion-like field on an n^3 grid, float32 torch tensor in [0, 1].

    F(p) = max_s 1/2 (1 - tanh((|p - c_s| - r_s(p)) / w_s)) with noisy radii
    r_s(p) = r_s (1 + radius_jitter * g(p)) (g a standardised spectral field),
    plus background * (B - mean B) with B a spectral field; then min-max.
    Radii scale with n / 1024 so that the geometry is size-independent.
    """
    import torch

    rng = np.random.default_rng(seed)
    scale = n / 1024.0
    centers = rng.uniform(0, n - 1, size=(n_spheres, 3))
    radii = rng.uniform(radius_range[0], radius_range[1], size=n_spheres) * scale
    widths = rng.uniform(width_range[0], width_range[1], size=n_spheres)
    g = spectral_field((n, n, n), seed + 101, device=device, normalize="std")
    out = torch.empty((n, n, n), device=device, dtype=torch.float32)
    ar = torch.arange(n, device=device, dtype=torch.float32)
    chunk = max(1, (1 << 24) // (n * n))
    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        zs = ar[z0:z1][:, None, None]
        jit = 1.0 + radius_jitter * g[z0:z1]
        best = torch.zeros((z1 - z0, n, n), device=device, dtype=torch.float32)
        for s in range(n_spheres):
            cx, cy, cz = (float(v) for v in centers[s])
            dist = torch.sqrt((ar[None, None, :] - cx) ** 2 + (ar[None, :, None] - cy) ** 2
                              + (zs - cz) ** 2)
            f = 0.5 * (1.0 - torch.tanh((dist - float(radii[s]) * jit) / float(widths[s])))
            torch.maximum(best, f, out=best)
        out[z0:z1] = best
    del g
    b = spectral_field((n, n, n), seed + 202, device=device, normalize="minmax")
    out += background * (b - b.mean())
    del b
    return minmax01(out).contiguous()


def field_stats(field):
    """Occupancy (V > 0.02) and the share of gradient magnitude in the top 10%.

    Comparable in kind to the structure statistics the paper tabulates for its
    datasets; central differences in the interior.
    """
    f = np.asarray(field, dtype=np.float64)
    occ = float(np.mean(f > 0.02))
    gz, gy, gx = np.gradient(f)
    g = np.sqrt(gx * gx + gy * gy + gz * gz).ravel()
    g.sort()
    top = g[int(0.9 * g.size):].sum() / max(g.sum(), 1e-300)
    return {"occupancy": occ, "top10_grad_share": float(top)}


def spectrum_slope(field, kmin=2.0, kmax=None):
    """Least-squares slope of log shell-energy vs log k (for fixture checks)."""
    f = np.asarray(field, dtype=np.float64)
    f = f - f.mean()
    n = f.shape[0]
    F = np.fft.fftn(f)
    e = np.abs(F) ** 2
    k = np.sqrt(sum(np.meshgrid(*[np.fft.fftfreq(s, 1.0 / s) ** 2 for s in f.shape],
                                indexing="ij")))
    kmax = kmax or n / 4
    kb = np.round(k).astype(int)
    ks = np.arange(int(kmin), int(kmax) + 1)
    E = np.array([e[kb == kk].sum() for kk in ks])
    slope = np.polyfit(np.log(ks), np.log(E), 1)[0]
    return float(slope)


def count_to_budget(shape, n):
    """Mean primitive spacing in voxels for a budget n on a grid of ``shape``."""
    return (float(np.prod(shape)) / n) ** (1.0 / 3.0)


def mixture_field_torch(params, shape, device="cpu", noise=0.0, seed=0, reach=6.0, chunk=128):
    """``mixture_field`` for large grids, in torch (float32 result).

    Each Gaussian is summed over the cube of half-width ceil(reach * max scale)
    voxels around its centre; beyond ``reach`` standard deviations along the
    longest axis a term is below exp(-reach^2 / 2) (1.5e-8 |c| at 6), so the
    sum equals the untruncated one to that level.  White noise of standard
    deviation ``noise`` is drawn from a torch generator seeded with ``seed``.
    """
    import torch

    nz, ny, nx = shape
    p = torch.as_tensor(np.asarray(params, dtype=np.float64), device=device)
    n = p.shape[1]
    q = p[3:7] / torch.linalg.norm(p[3:7], dim=0, keepdim=True)
    w, x, y, z = q
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]),
    ]).permute(2, 0, 1)                                      # [n, 3, 3]
    inv_s = torch.exp(-p[7:10]).T                           # [n, 3]
    h = int(np.ceil(reach * float(torch.exp(p[7:10]).max())))
    o = torch.arange(-h, h + 1, device=device, dtype=torch.float64)
    oz, oy, ox = torch.meshgrid(o, o, o, indexing="ij")
    offs = torch.stack([ox.ravel(), oy.ravel(), oz.ravel()], dim=1)      # [C, 3]
    out = torch.zeros(nz * ny * nx, device=device, dtype=torch.float64)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        mu = p[0:3, a:b].T                                   # [m, 3]
        base = torch.floor(mu)
        pts = base[:, None, :] + offs[None]                  # [m, C, 3]
        d = pts - mu[:, None, :]
        zloc = torch.einsum("mcj,mjk->mck", d, R[a:b]) * inv_s[a:b, None, :]
        val = p[10, a:b, None] * torch.exp(-0.5 * (zloc * zloc).sum(-1))
        ix, iy, iz = pts[..., 0].long(), pts[..., 1].long(), pts[..., 2].long()
        ok = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny) & (iz >= 0) & (iz < nz)
        idx = (ix + nx * (iy + ny * iz))[ok]
        out.index_add_(0, idx, val[ok])
    if noise > 0:
        gen = torch.Generator(device=device).manual_seed(int(seed))
        out += noise * torch.randn(out.shape, generator=gen, device=device, dtype=torch.float64)
    return out.reshape(nz, ny, nx).to(torch.float32)


# Allowed edge lengths and the voxel cap of the batched workload.
BATCH_DIMS = tuple(range(96, 385, 32))
BATCH_MAX_VOXELS = 512 * 256 * 128


def batch_shapes(count, seed):
    """``count`` grid shapes (nz, ny, nx), each edge drawn from BATCH_DIMS and
    redrawn until the volume holds at most BATCH_MAX_VOXELS voxels."""
    rng = np.random.default_rng(seed)
    shapes = []
    while len(shapes) < count:
        d = rng.choice(BATCH_DIMS, size=3)
        if int(np.prod(d)) <= BATCH_MAX_VOXELS:
            shapes.append(tuple(int(v) for v in d))
    return shapes


def batch_item_field(shape, seed, device="cpu"):
    """Volume ``seed`` of the batched workload, normalised to [0, 1]: even seeds
    are signed Gaussian mixtures (200 per 64^3 of volume, scales 1-4 voxels,
    weights U[-1, 1], noise 0.01), odd seeds k^-5/3 spectral fields."""
    nz, ny, nx = shape
    if seed % 2 == 0:
        count = max(1, int(round(200 * nz * ny * nx / 64 ** 3)))
        params = random_params(count, (nx, ny, nz), seed)
        f = mixture_field_torch(params, shape, device=device, noise=0.01, seed=seed)
        return minmax01(f).contiguous()
    return spectral_field(shape, seed, device=device)


def gradient_energy(field):
    """sum |grad V|^2 with central differences (one-sided at the faces)."""
    import torch

    gz, gy, gx = torch.gradient(field.to(torch.float64))
    return float((gx * gx + gy * gy + gz * gz).sum())


def batch_budgets(energies, lo=8000, hi=200000):
    """Budgets proportional to the gradient energy: hi * E / max E, within [lo, hi]."""
    e = np.asarray(energies, dtype=np.float64)
    return [int(v) for v in np.clip(np.round(hi * e / e.max()), lo, hi)]
