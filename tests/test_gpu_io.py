"""Export (Sec. III-I; Sec. III-J eq:size) and checkpoint/resume on the device library.

The export is checked field by field against the parameters it was written
from (its layout: twelve float32 per primitive, position, log-scale,
quaternion w x y z, attribute a = c, weight w = 1, after a fixed header), and
its size against the oracle's 48 N + H.  Resuming from a checkpoint and
refining must give bitwise the parameters of an uninterrupted run (gradient
sums are deterministic), so the check is exact.
"""
import struct

import numpy as np
import pytest

from oracle import field as F
from synth import fields as S

pytestmark = pytest.mark.gpu


def _setup(n=700, seed=4):
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    grid = g.Grid(40, 36, 30, 2, -1, 5)
    ogrid = F.Grid(40, 36, 30, 2, -1, 5)
    theta = S.random_params(n, (40, 36, 30), seed=seed, scale_range=(0.6, 3.0))
    theta[0:3] += np.array([[2.0], [-1.0], [5.0]])       # world coordinates of the grid
    gen = S.random_params(60, (40, 36, 30), seed=seed + 1, scale_range=(1.0, 4.0))
    V = S.mixture_field(gen, ogrid.shape)
    return g, torch, grid, theta.astype(np.float32), torch.from_numpy(V.astype(np.float32)).cuda()


def test_export_layout_size_and_roundtrip():
    g, torch, grid, theta, V = _setup()
    ctx = g.Context(k=3.0)
    P = g.Params(ctx, theta.shape[1]).upload(theta)
    buf = g.export_bytes(ctx, P, grid, vmin=-0.5, vmax=2.0)
    n = theta.shape[1]
    assert len(buf) == F.encoded_bytes(n, g.EXPORT_HEADER)
    assert buf[:4] == b"GVE1"
    version, nn = struct.unpack_from("<Iq", buf, 4)
    assert version == 1 and nn == n
    assert struct.unpack_from("<6q", buf, 16) == (40, 36, 30, 2, -1, 5)
    k, vmin, vmax = struct.unpack_from("<3f", buf, 64)
    assert (k, vmin, vmax) == (3.0, -0.5, 2.0)
    rec = np.frombuffer(buf, dtype=np.float32, offset=g.EXPORT_HEADER).reshape(n, 12)
    assert np.array_equal(rec[:, 0:3], theta[0:3].T)
    assert np.array_equal(rec[:, 3:6], theta[7:10].T)
    assert np.array_equal(rec[:, 6:10], theta[3:7].T)
    assert np.array_equal(rec[:, 10], theta[10]) and np.all(rec[:, 11] == 1.0)
    lut = np.frombuffer(buf, dtype=np.float32, offset=256, count=1024).reshape(256, 4)
    assert np.allclose(lut[:, 0], np.arange(256) / 255.0) and np.all(np.diff(lut[:, 3]) > 0)
    Q, g2 = g.import_bytes(ctx, buf)
    assert (g2.nx, g2.ny, g2.nz, g2.x0, g2.y0, g2.z0) == (40, 36, 30, 2, -1, 5)
    assert np.array_equal(Q.download(), theta) and Q.step == 0
    a = g.evaluate(ctx, P, grid).cpu().numpy()
    b = g.evaluate(ctx, Q, grid).cpu().numpy()
    assert np.array_equal(a, b)


def test_import_weight_scales_attribute_and_rejects_malformed():
    g, torch, grid, theta, V = _setup(n=50)
    ctx = g.Context()
    P = g.Params(ctx, 50).upload(theta)
    buf = bytearray(g.export_bytes(ctx, P, grid))
    rec = np.frombuffer(buf, dtype=np.float32, offset=g.EXPORT_HEADER).reshape(50, 12)
    rec = rec.copy()
    rec[:, 10] = 2.0
    rec[:, 11] = theta[10] / 2.0
    buf[g.EXPORT_HEADER:] = rec.tobytes()
    Q, _ = g.import_bytes(ctx, bytes(buf))
    assert np.allclose(Q.download()[10], theta[10], rtol=1e-7, atol=0)
    with pytest.raises(g.GveError):
        g.import_bytes(ctx, b"XXXX" + bytes(buf[4:]))
    with pytest.raises(g.GveError):
        g.import_bytes(ctx, bytes(buf[:-4]))
    with pytest.raises(g.GveError):
        g.import_bytes(ctx, bytes(buf[:100]))


@pytest.mark.parametrize("deterministic", [True])
def test_resume_from_checkpoint_is_bitwise(deterministic):
    g, torch, grid, theta, V = _setup()
    ctx = g.Context(k=3.0, lr=5e-3, deterministic=deterministic)
    A = g.Params(ctx, theta.shape[1]).upload(theta)
    la = g.refine(ctx, A, V, grid, 12)
    B = g.Params(ctx, theta.shape[1]).upload(theta)
    lb1 = g.refine(ctx, B, V, grid, 5)
    ck = g.checkpoint_bytes(ctx, B, elapsed_s=12.5)
    B.close()
    C, el = g.checkpoint_load(ctx, ck)
    assert el == 12.5 and C.step == 5
    lb2 = g.refine(ctx, C, V, grid, 7)
    assert np.array_equal(np.concatenate([lb1, lb2]), la)
    assert np.array_equal(C.download(), A.download())
    with pytest.raises(g.GveError):
        g.checkpoint_load(ctx, ck[:-1])
