"""The rate probes return physically possible rates for one MI355X (each
below the published peak of its unit, with a small allowance for clock
boost) and the fused kernel's measured work fits within them."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_rates_are_plausible():
    import torch

    import paper_2608_14112_amd as g
    assert torch.cuda.is_available()
    ctx = g.Context()
    r = g.probe(ctx)
    print(r, flush=True)
    # fp32 vector peak 157.3 TFLOP/s (the probe issues non-packed FMAs)
    assert 1e12 < r["fma_flops_per_s"] <= 1.1 * 157.3e12
    # transcendental: at most one per FMA lane-slot (78.6e12 per second)
    assert 1e11 < r["exp_per_s"] <= 1.1 * 78.65e12
    # HBM3E: 8 TB/s
    assert 1e11 < r["copy_bytes_per_s"] <= 1.1 * 8e12
    assert 1e7 < r["atomic_instr_per_s"] < 1e12
