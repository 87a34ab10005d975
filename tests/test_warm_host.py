"""Host logic of the warm-started time-to-PSNR run (no GPU needed): the size
of each refinement call after the first."""
import math

import numpy as np


def test_next_call_size_lands_on_the_target():
    from paper_2608_14112_amd.warm import next_call_size

    # geometric decrease by e^-0.01 per iteration; the previous call recorded
    # the states after 0 .. 63 of its updates and made all 64
    losses = 1000.0 * np.exp(-0.01 * np.arange(64))
    target = 1000.0 * math.exp(-0.01 * 100)       # reached 100 updates into that call
    size, rate = next_call_size(losses, target, None, 64)
    assert math.isclose(rate, 0.01, rel_tol=1e-9)
    # a call of 37 records the states after 64 .. 100 updates: the target at its end
    assert size == 37
    # at most `most`, at least one
    assert next_call_size(losses, 1e-30, None, 64)[0] == 64
    assert next_call_size(losses, losses[-1] * 0.999, None, 64)[0] == 1


def test_next_call_size_keeps_the_last_rate_and_falls_back():
    from paper_2608_14112_amd.warm import next_call_size

    # one recorded loss: the previous rate is kept
    assert next_call_size(np.array([5.0]), 1.0, 0.01, 64) == (64, 0.01)
    size, rate = next_call_size(np.array([math.e]), 1.0, 0.1, 64)
    assert rate == 0.1 and size == 10                 # log(e / 1) / 0.1 updates
    # no decrease seen and no earlier rate: the largest call
    assert next_call_size(np.array([2.0, 2.0, 2.0]), 1.0, None, 32) == (32, None)
    assert next_call_size(np.array([1.0, 2.0]), 0.5, None, 16) == (16, None)


def test_next_call_size_with_non_finite_losses():
    from paper_2608_14112_amd.warm import next_call_size

    assert next_call_size(np.array([2.0, np.inf]), 1.0, 0.01, 16) == (16, 0.01)
    assert next_call_size(np.array([2.0, np.nan]), 1.0, 0.01, 16) == (16, 0.01)
    assert next_call_size(np.array([np.nan, 1.5]), 1.0, None, 16) == (16, None)
