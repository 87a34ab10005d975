"""A context gives back every device buffer it grew when it is destroyed.

Each cycle creates a context, runs the calls that grow the most kinds of
workspace buffer (binning with deterministic gradient slots, the dense
reference path's residual), and destroys it; the device's free memory must
not keep falling from cycle to cycle.
"""
import numpy as np
import pytest

from synth import fields as S

pytestmark = pytest.mark.gpu


def test_destroy_frees_the_workspace():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    n_side, n = 96, 3000
    grid = g.Grid(n_side, n_side, n_side)
    theta = S.random_params(n, n_side, seed=3, scale_range=(1.0, 3.0)).astype(np.float32)
    field = torch.rand((n_side, n_side, n_side), device="cuda", dtype=torch.float32)
    grad = torch.empty((11, n), device="cuda", dtype=torch.float32)

    def cycle():
        ctx = g.Context(deterministic=True)
        P = g.Params(ctx, n).upload(theta)
        g.loss_grad(ctx, P, field, grid, grad)
        g.dense_loss_grad(ctx, P, field, grid, grad)
        torch.cuda.synchronize()
        ws = ctx.stats()["workspace_bytes"]
        P.close()
        ctx.close()
        torch.cuda.synchronize()
        return ws

    ws = cycle()                      # first cycle: library and torch warm up
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        cycle()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"workspace {ws / 1e6:.1f} MB per context, free memory change "
          f"{(free1 - free0) / 1e6:.1f} MB over 5 cycles", flush=True)
    assert ws > 4 * n_side ** 3       # the dense residual alone is M floats
    # a leak of the workspace would lose 5 x ws
    assert free0 - free1 < ws


def test_package_imported_before_torch_shares_its_hip_runtime():
    """A program that imports the package before torch gets one HIP runtime
    (torch's), and a context works on torch's tensors: run in a fresh process,
    since this one has imported torch already."""
    import os
    import subprocess
    import sys

    code = """
import paper_2608_14112_amd as g
import numpy as np
import torch
from synth import fields as S
hip = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}
assert len(hip) == 1, hip
ctx = g.Context()
grid = g.Grid(32, 32, 32)
P = g.Params(ctx, 200).upload(S.random_params(200, 32, seed=5).astype(np.float32))
out = g.evaluate(ctx, P, grid)
torch.cuda.synchronize()
assert torch.isfinite(out).all() and float(out.abs().sum()) > 0
print('one runtime:', hip.pop(), flush=True)
"""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=300)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0
